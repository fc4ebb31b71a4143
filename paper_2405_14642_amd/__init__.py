"""Batched midsize big-integer arithmetic on MI355X (gfx950).

Thin Python binding over the C ABI in ``include/bigint.h`` (library
``libbigint.so`` next to this file).  It only marshals arguments: every step
of addition and multiplication runs in the library's HIP kernels.  Device
memory and streams come from PyTorch (tensors are used as raw limb buffers).

The names follow the C ABI: ``bigadd``, ``bigmul``, ``bigadd_v``,
``bigmul_v``, ``fused`` (``bi_fused``); ``Context`` wraps ``bi_ctx``.
"""
from __future__ import annotations

import ctypes
import os

__all__ = ["Context", "BigIntError", "bigadd", "bigmul", "bigadd_v", "bigmul_v", "fused", "ntt_field", "StreamQueue",
           "DESC_DTYPE", "lib", "library_path",
           "MUL_AUTO", "MUL_SCHOOL_VALU", "MUL_SCHOOL_MFMA", "MUL_NTT", "MUL_NTT_PF64", "MUL_KARATSUBA", "PROG_ADD6", "PROG_POLY", "PROG_MUL_LOW", "MAX_BITS",
           "STATUS"]

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libbigint.so")

MUL_AUTO, MUL_SCHOOL_VALU, MUL_SCHOOL_MFMA, MUL_NTT, MUL_NTT_PF64, MUL_KARATSUBA = 0, 1, 2, 3, 4, 5
PROG_ADD6, PROG_POLY, PROG_MUL_LOW = 1, 2, 3
MAX_BITS = 1 << 18
STATUS = {0: "BI_OK", -1: "BI_EINVAL", -2: "BI_ESIZE", -3: "BI_ELIMB", -4: "BI_EALIAS", -5: "BI_EHIP",
          -6: "BI_ENOMEM", -7: "BI_EALGO", -8: "BI_ENODEV"}

EXPORTS = ("bi_ctx_create", "bi_ctx_destroy", "bi_status_str", "bi_last_error",
           "bigadd", "bigmul", "bigadd_v", "bigmul_v", "bi_ntt_field", "bi_autotune", "bi_tune_get",
           "bi_tune_set", "bi_stream_open", "bi_stream_submit", "bi_stream_poll", "bi_stream_wait",
           "bi_stream_close", "bi_fused", "bi_tune_get_valu",
           "bi_tune_set_valu", "bigadd_large", "bigmul_large", "bi_tune_save",
           "bi_tune_load", "bi_mul_plan", "bigmul_noalloc", "bi_tune_get_kara", "bi_tune_set_kara",
           "bi_tune_get_list", "bi_tune_set_list", "bi_mul_large_plan")
NUM_CLASSES = 10


class NttFieldInfo(ctypes.Structure):
    """bi_ntt_field_info: p = k 2^two_adicity + 1, g = a^k a primitive
    2^two_adicity-th root of unity (Section 4.1)."""
    _fields_ = [("p", ctypes.c_uint64), ("k", ctypes.c_uint64), ("two_adicity", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("a", ctypes.c_uint64), ("g", ctypes.c_uint64)]


class MulPlanInfo(ctypes.Structure):
    """bi_mul_plan_info: the algorithm bigmul runs, and for Karatsuba its
    levels, base product size (32-bit words) and base algorithm."""
    _fields_ = [("algo", ctypes.c_int), ("kara_levels", ctypes.c_int), ("base_limbs", ctypes.c_uint32),
                ("base_algo", ctypes.c_int)]


class BigIntError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        self.name = STATUS.get(status, str(status))
        super().__init__(f"{self.name}: {message}")


def _load():
    # PyTorch ships its own HIP runtime (libamdhip64, same SONAME as the one
    # in /opt/rocm).  Loading torch first makes libbigint.so bind to that
    # already-loaded runtime, so the process holds exactly one HIP runtime and
    # the tensors and streams torch hands us are valid for our launches.
    import torch  # noqa: F401

    if not os.path.exists(library_path):
        raise ImportError(f"{library_path} is missing: the HIP library has not been built "
                          "(run __graft_entry__.build() or python -m paper_2405_14642_amd.build)")
    L = ctypes.CDLL(library_path)
    P, U32, U64, I = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    L.bi_ctx_create.argtypes = [I, ctypes.POINTER(P)]
    L.bi_ctx_destroy.argtypes = [P]
    L.bi_ctx_destroy.restype = None
    L.bi_status_str.argtypes = [I]
    L.bi_status_str.restype = ctypes.c_char_p
    L.bi_last_error.argtypes = []
    L.bi_last_error.restype = ctypes.c_char_p
    L.bigadd.argtypes = [P, P, P, P, P, U32, U32, U64, P]
    L.bigmul.argtypes = [P, P, P, P, U32, U32, U64, I, P]
    L.bigmul_noalloc.argtypes = [P, P, P, P, U32, U32, U64, I, P]
    L.bigadd_large.argtypes = [P, P, P, P, P, U64, U32, P]
    L.bigmul_large.argtypes = [P, P, P, P, U64, U32, I, U32, P]
    L.bigadd_v.argtypes = [P, P, P, P, P, P, U64, U32, P]
    L.bigmul_v.argtypes = [P, P, P, P, P, U64, U32, I, P]
    L.bi_ntt_field.argtypes = [U64, P]
    L.bi_autotune.argtypes = [P, P, P, U32]
    L.bi_tune_get.argtypes = [P, P, U32]
    L.bi_tune_set.argtypes = [P, P, U32]
    L.bi_tune_save.argtypes = [P, ctypes.c_char_p]
    L.bi_tune_load.argtypes = [P, ctypes.c_char_p]
    L.bi_stream_open.argtypes = [P, P, U64, P, U64, P, U64, U32, U64, I, I, P, ctypes.POINTER(P)]
    L.bi_stream_submit.argtypes = [P, P, U64, ctypes.POINTER(U64)]
    L.bi_stream_poll.argtypes = [P, U64, ctypes.POINTER(I)]
    L.bi_stream_wait.argtypes = [P, U64]
    L.bi_stream_close.argtypes = [P]
    L.bi_fused.argtypes = [P, I, P, P, P, U32, U32, U64, P]
    L.bi_tune_get_valu.argtypes = [P, P, P, U32]
    L.bi_tune_set_valu.argtypes = [P, P, P, U32]
    L.bi_mul_plan.argtypes = [P, U32, U32, I, P]
    L.bi_mul_large_plan.argtypes = [U64, U32, I, ctypes.POINTER(U32), ctypes.POINTER(U32)]
    L.bi_tune_get_list.argtypes = [P, P, U32]
    L.bi_tune_set_list.argtypes = [P, P, U32]
    L.bi_tune_get_kara.argtypes = [P, P, U32]
    L.bi_tune_set_kara.argtypes = [P, P, U32]
    for f in (L.bi_mul_large_plan, L.bi_tune_get_list, L.bi_tune_set_list, L.bi_tune_get_kara, L.bi_tune_set_kara, L.bi_mul_plan, L.bigmul_noalloc, L.bi_ctx_create, L.bigadd, L.bigmul, L.bigadd_v, L.bigmul_v, L.bi_ntt_field, L.bi_autotune,
              L.bi_tune_get, L.bi_tune_set, L.bi_stream_open, L.bi_stream_submit, L.bi_stream_poll,
              L.bi_stream_wait, L.bi_stream_close, L.bi_fused, L.bi_tune_get_valu,
              L.bi_tune_set_valu, L.bigadd_large, L.bigmul_large, L.bi_tune_save, L.bi_tune_load):
        f.restype = I
    return L


lib = _load()


def _check(st: int):
    if st != 0:
        raise BigIntError(st, lib.bi_last_error().decode())


def _ptr(x):
    """Device address of a tensor, an int address, or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream, ref=None):
    if stream is not None:
        return stream if isinstance(stream, int) else stream.cuda_stream
    import torch
    dev = ref.device if ref is not None and hasattr(ref, "device") else None
    return torch.cuda.current_stream(dev).cuda_stream


def _require(*args):
    """Host-side check of the tensor arguments before any library call:
    each (name, tensor, bytes needed[, element width]) must be contiguous,
    hold at least that many bytes, have elements of that width when given,
    and (checked last, for all of them) live on the GPU.  Plain int
    addresses and None are passed through unchecked."""
    ts = [x for x in args if x[1] is not None and not isinstance(x[1], int)]
    for name, t, nbytes, *width in ts:
        have = t.numel() * t.element_size()
        if width and width[0] is not None and t.element_size() != width[0]:
            raise ValueError(f"{name} has {t.element_size()}-byte elements, the other operands {width[0]}-byte ones")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if have < nbytes:
            raise ValueError(f"{name} holds {have} bytes, the call needs {nbytes}")
    for name, t, *_ in ts:
        if not t.is_cuda:
            raise ValueError(f"{name} must be a device tensor")


def _width(t):
    return None if t is None or isinstance(t, int) else t.element_size()


def _limb_bits(t, limb_bits):
    if limb_bits is not None:
        return limb_bits
    size = t.element_size()
    if size not in (4, 8):
        raise ValueError("limb tensors must have 4- or 8-byte elements")
    return 8 * size


class Context:
    """A library context (bi_ctx) on one HIP device."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        _check(lib.bi_ctx_create(device, ctypes.byref(h)))
        self.handle = h.value
        self.device = device

    def close(self):
        if self.handle:
            lib.bi_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def _h(ctx):
    return None if ctx is None else (ctx if isinstance(ctx, int) else ctx.handle)


def bigadd(ctx, a, b, out, carry=None, n_limbs=None, limb_bits=None, batch=None, stream=None):
    """out = a + b per instance (and carry bytes).  Tensors are (batch, n) limb arrays."""
    lb = _limb_bits(a, limb_bits)
    n = n_limbs if n_limbs is not None else a.shape[-1]
    bt = batch if batch is not None else (a.numel() // n if n else 0)
    w, nb = _width(a), n * bt * lb // 8
    _require(("a", a, nb, w), ("b", b, nb, w), ("out", out, nb, w), ("carry", carry, bt))
    _check(lib.bigadd(_h(ctx), _ptr(a), _ptr(b), _ptr(out), _ptr(carry), n, lb, bt, _stream(stream, a)))
    return out


def bigadd_large(ctx, a, b, out, carry=None, n_limbs=None, limb_bits=None, stream=None):
    """out = a + b for ONE integer of any length (1-D limb tensors); carry is
    a one-byte device tensor or None."""
    lb = _limb_bits(a, limb_bits)
    n = n_limbs if n_limbs is not None else a.numel()
    w, nb = _width(a), n * lb // 8
    _require(("a", a, nb, w), ("b", b, nb, w), ("out", out, nb, w), ("carry", carry, 1))
    _check(lib.bigadd_large(_h(ctx), _ptr(a), _ptr(b), _ptr(out), _ptr(carry), n, lb, _stream(stream, a)))
    return out


def bigmul_large(ctx, a, b, out, algo=MUL_AUTO, block_bits=0, n_limbs=None, limb_bits=None, stream=None):
    """out (2n limbs) = a * b for ONE pair of integers beyond 2^18 bits (1-D
    limb tensors); algo and block_bits (0 = by size, else 2^16..2^18) pick
    the block products."""
    lb = _limb_bits(a, limb_bits)
    n = n_limbs if n_limbs is not None else a.numel()
    w, nb = _width(a), n * lb // 8
    _require(("a", a, nb, w), ("b", b, nb, w), ("out", out, 2 * nb, w))
    _check(lib.bigmul_large(_h(ctx), _ptr(a), _ptr(b), _ptr(out), n, lb, int(algo), int(block_bits),
                            _stream(stream, a)))
    return out


def bigmul(ctx, a, b, out, algo=MUL_AUTO, n_limbs=None, limb_bits=None, batch=None, stream=None):
    """out (batch, 2n) = a * b per instance."""
    lb = _limb_bits(a, limb_bits)
    n = n_limbs if n_limbs is not None else a.shape[-1]
    bt = batch if batch is not None else (a.numel() // n if n else 0)
    w, nb = _width(a), n * bt * lb // 8
    _require(("a", a, nb, w), ("b", b, nb, w), ("out", out, 2 * nb, w))
    _check(lib.bigmul(_h(ctx), _ptr(a), _ptr(b), _ptr(out), n, lb, bt, int(algo), _stream(stream, a)))
    return out


def bigmul_noalloc(ctx, a, b, out, algo=MUL_AUTO, n_limbs=None, limb_bits=None, batch=None, stream=None):
    """bigmul with every scratch buffer in the library's fixed per-GPU array
    (no device allocation; calls on one GPU must not overlap in time)."""
    lb = _limb_bits(a, limb_bits)
    n = n_limbs if n_limbs is not None else a.shape[-1]
    bt = batch if batch is not None else (a.numel() // n if n else 0)
    w, nb = _width(a), n * bt * lb // 8
    _require(("a", a, nb, w), ("b", b, nb, w), ("out", out, 2 * nb, w))
    _check(lib.bigmul_noalloc(_h(ctx), _ptr(a), _ptr(b), _ptr(out), n, lb, bt, int(algo), _stream(stream, a)))
    return out


def fused(ctx, program, a, b, out, n_limbs=None, limb_bits=None, batch=None, stream=None):
    """out (batch, n) = the fused program (PROG_ADD6: 4a + 3b; PROG_POLY:
    (a a + b)(b b + b) + a b; PROG_MUL_LOW: a b), mod 2^(n * limb_bits) per
    instance."""
    lb = _limb_bits(a, limb_bits)
    n = n_limbs if n_limbs is not None else a.shape[-1]
    bt = batch if batch is not None else (a.numel() // n if n else 0)
    w, nb = _width(a), n * bt * lb // 8
    _require(("a", a, nb, w), ("b", b, nb, w), ("out", out, nb, w))
    _check(lib.bi_fused(_h(ctx), int(program), _ptr(a), _ptr(b), _ptr(out), n, lb, bt, _stream(stream, a)))
    return out


def bigadd_v(ctx, a, b, out, carry, desc, count, limb_bits, stream=None):
    """Ragged addition; desc is a device buffer of `count` bi_desc records
    (uint64 a_off, b_off, out_off; uint32 n_limbs, reserved)."""
    _require(("desc", desc, 32 * count), ("carry", carry, count))
    _check(lib.bigadd_v(_h(ctx), _ptr(a), _ptr(b), _ptr(out), _ptr(carry), _ptr(desc), count, limb_bits,
                        _stream(stream, a)))
    return out


def autotune(ctx, stream=None):
    """Time every algorithm per size class on the device; returns the chosen
    algorithm per class (list of NUM_CLASSES ints)."""
    out = (ctypes.c_int * NUM_CLASSES)()
    _check(lib.bi_autotune(_h(ctx), _stream(stream), out, NUM_CLASSES))
    return list(out)


def tune_get(ctx):
    out = (ctypes.c_int * NUM_CLASSES)()
    _check(lib.bi_tune_get(_h(ctx), out, NUM_CLASSES))
    return list(out)


def mul_plan(ctx, n_limbs, limb_bits=32, algo=MUL_AUTO):
    """What bigmul runs for n_limbs-limb operands: dict(algo, kara_levels,
    base_limbs, base_algo)."""
    info = MulPlanInfo()
    _check(lib.bi_mul_plan(_h(ctx), n_limbs, limb_bits, algo, ctypes.byref(info)))
    return {k: getattr(info, k) for k, _ in MulPlanInfo._fields_}


def mul_large_plan(n_limbs, limb_bits=32, algo=MUL_AUTO):
    """(block_bits, blocks) bigmul_large picks by default."""
    bb, k = ctypes.c_uint32(), ctypes.c_uint32()
    _check(lib.bi_mul_large_plan(n_limbs, limb_bits, int(algo), ctypes.byref(bb), ctypes.byref(k)))
    return bb.value, k.value


def tune_get_list(ctx):
    """Ragged-batch algorithm per size class."""
    out = (ctypes.c_int * NUM_CLASSES)()
    _check(lib.bi_tune_get_list(_h(ctx), out, NUM_CLASSES))
    return list(out)


def tune_set_list(ctx, algos):
    arr = (ctypes.c_int * len(algos))(*algos)
    _check(lib.bi_tune_set_list(_h(ctx), arr, len(algos)))


def tune_get_kara(ctx):
    """Karatsuba base (32-bit words) per size class."""
    out = (ctypes.c_uint32 * NUM_CLASSES)()
    _check(lib.bi_tune_get_kara(_h(ctx), out, NUM_CLASSES))
    return list(out)


def tune_set_kara(ctx, bases):
    arr = (ctypes.c_uint32 * len(bases))(*bases)
    _check(lib.bi_tune_set_kara(_h(ctx), arr, len(bases)))


def tune_set(ctx, algos):
    arr = (ctypes.c_int * len(algos))(*algos)
    _check(lib.bi_tune_set(_h(ctx), arr, len(algos)))


def tune_save(ctx, path):
    """Write the context's tuning tables to `path` (keyed by architecture
    and HIP runtime version)."""
    _check(lib.bi_tune_save(_h(ctx), os.fsencode(path)))


def tune_load(ctx, path):
    """Load tuning tables written by tune_save for this architecture and
    runtime version (BigIntError otherwise; nothing changed)."""
    _check(lib.bi_tune_load(_h(ctx), os.fsencode(path)))


def tune_get_valu(ctx):
    """The VALU schoolbook schedule per class: list of (Q, waves), (0, 0)
    where the built-in size rule applies."""
    q = (ctypes.c_int * NUM_CLASSES)()
    w = (ctypes.c_int * NUM_CLASSES)()
    _check(lib.bi_tune_get_valu(_h(ctx), q, w, NUM_CLASSES))
    return list(zip(list(q), list(w)))


def tune_set_valu(ctx, schedule):
    """Set the VALU schoolbook schedule per class from a list of (Q, waves)
    pairs ((0, 0): the built-in size rule)."""
    q = (ctypes.c_int * len(schedule))(*[int(x[0]) for x in schedule])
    w = (ctypes.c_int * len(schedule))(*[int(x[1]) for x in schedule])
    _check(lib.bi_tune_set_valu(_h(ctx), q, w, len(schedule)))


def ntt_field(p: int) -> NttFieldInfo:
    """Host-side prime-field search of Section 4.1 (no GPU needed)."""
    info = NttFieldInfo()
    _check(lib.bi_ntt_field(p, ctypes.byref(info)))
    return info


def bigmul_v(ctx, a, b, out, desc, count, limb_bits, algo=MUL_AUTO, stream=None):
    """Ragged multiplication; desc as for bigadd_v (results of 2 n_limbs limbs)."""
    _require(("desc", desc, 32 * count))
    _check(lib.bigmul_v(_h(ctx), _ptr(a), _ptr(b), _ptr(out), _ptr(desc), count, limb_bits, int(algo),
                        _stream(stream, a)))
    return out


def _desc_dtype():
    import numpy as np
    return np.dtype([("a_off", "<u8"), ("b_off", "<u8"), ("out_off", "<u8"), ("n_limbs", "<u4"),
                     ("reserved", "<u4")])


DESC_DTYPE = _desc_dtype()


class StreamQueue:
    """bi_stream: bursts of ragged products over fixed operand buffers.

    ``submit`` takes a host numpy array of DESC_DTYPE records and returns a
    ticket; ``poll`` / ``wait`` report its completion."""

    def __init__(self, ctx, a, b, out, limb_bits, max_descs, algo=MUL_AUTO, use_graph=True, stream=None):
        q = ctypes.c_void_p()
        self._keep = (ctx, a, b, out)
        _check(lib.bi_stream_open(_h(ctx), _ptr(a), a.numel() * a.element_size() * 8 // limb_bits, _ptr(b),
                                  b.numel() * b.element_size() * 8 // limb_bits, _ptr(out),
                                  out.numel() * out.element_size() * 8 // limb_bits, limb_bits, max_descs,
                                  int(algo), 1 if use_graph else 0, _stream(stream, a), ctypes.byref(q)))
        self.handle = q.value

    def submit(self, descs) -> int:
        import numpy as np
        d = np.ascontiguousarray(descs, dtype=DESC_DTYPE)
        t = ctypes.c_uint64()
        _check(lib.bi_stream_submit(self.handle, d.ctypes.data, len(d), ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int) -> bool:
        done = ctypes.c_int()
        _check(lib.bi_stream_poll(self.handle, ticket, ctypes.byref(done)))
        return bool(done.value)

    def wait(self, ticket: int):
        _check(lib.bi_stream_wait(self.handle, ticket))

    def close(self):
        if self.handle:
            h, self.handle = self.handle, None
            _check(lib.bi_stream_close(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
