"""Helpers for the GPU tests: numpy limb arrays <-> device tensors, descriptors."""
from __future__ import annotations

import numpy as np

_IDT = {np.dtype(np.uint32): np.int32, np.dtype(np.uint64): np.int64}


def to_dev(x: np.ndarray):
    import torch
    x = np.ascontiguousarray(x)
    return torch.from_numpy(x.view(_IDT[x.dtype])).to("cuda")


def empty_dev(shape, dtype):
    import torch
    tdt = torch.int32 if np.dtype(dtype) == np.uint32 else torch.int64
    return torch.empty(shape, dtype=tdt, device="cuda")


def zeros_u8(n):
    import torch
    return torch.zeros(n, dtype=torch.uint8, device="cuda")


def from_dev(t, dtype) -> np.ndarray:
    return t.cpu().numpy().view(dtype)


DESC_DTYPE = np.dtype([("a_off", "<u8"), ("b_off", "<u8"), ("out_off", "<u8"), ("n_limbs", "<u4"),
                       ("reserved", "<u4")])


def desc_dev(a_off, b_off, out_off, n):
    import torch
    d = np.zeros(len(n), dtype=DESC_DTYPE)
    d["a_off"], d["b_off"], d["out_off"], d["n_limbs"] = a_off, b_off, out_off, n
    return torch.from_numpy(d.view(np.uint8).copy()).to("cuda")


def sync():
    import torch
    torch.cuda.synchronize()
