"""Parity of the HIP addition kernels with the CPU oracle (bit-exact)."""
from __future__ import annotations

import zlib

import numpy as np
import pytest

import workloads as W
from tests import gpu_util as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import paper_2405_14642_amd as B
    return B


@pytest.fixture(scope="module")
def ctx(B):
    c = B.Context(0)
    yield c
    c.close()


def run_add(B, ctx, a, b, in_place=None):
    A, Bt = G.to_dev(a), G.to_dev(b)
    out = {"a": A, "b": Bt}.get(in_place) if in_place else G.empty_dev(a.shape, a.dtype)
    carry = G.zeros_u8(a.shape[0])
    B.bigadd(ctx, A, Bt, out, carry)
    G.sync()
    return G.from_dev(out, a.dtype), carry.cpu().numpy()


def check(orc, a, b, got, carry):
    want, wc = orc.add(a, b)
    bad = np.nonzero((got != want).any(axis=1) | (carry != wc))[0]
    assert bad.size == 0, f"{bad.size} instances differ, first {bad[:8]}"


def rand(rng, batch, n, dt):
    return rng.integers(0, np.iinfo(dt).max, size=(batch, n), dtype=dt, endpoint=True)


def test_small_workload(B, ctx, orc):
    a, b = W.small_inputs()
    got, carry = run_add(B, ctx, a, b)
    check(orc, a, b, got, carry)


@pytest.mark.parametrize("dt", [np.uint32, np.uint64])
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 7, 8, 15, 16, 17, 31, 32, 33, 63, 64, 65, 100, 127, 128, 129,
                               255, 256, 257, 1000, 1024, 4095, 4096])
def test_sizes_and_tails(B, ctx, orc, n, dt):
    if n * np.dtype(dt).itemsize * 8 > W.MAX_BITS:
        pytest.skip("beyond the size limit")
    rng = np.random.default_rng(n * 7 + np.dtype(dt).itemsize)
    batch = 67  # not a multiple of any instances-per-row count
    a, b = rand(rng, batch, n, dt), rand(rng, batch, n, dt)
    mx = np.iinfo(dt).max
    a[::3] = mx                     # carry runs from the low limb to the top
    b[::3] = 0
    b[::3, 0] = 1
    a[1::5] = mx                    # carry starts at a random limb
    b[1::5, : max(1, n // 3)] = rand(rng, b[1::5].shape[0], max(1, n // 3), dt)
    b[1::5, max(1, n // 3):] = 0
    a[2::7], b[2::7] = mx, mx       # all-ones + all-ones
    got, carry = run_add(B, ctx, a, b)
    check(orc, a, b, got, carry)


def test_max_size_u32(B, ctx, orc):
    n = W.MAX_BITS // 32
    rng = np.random.default_rng(3)
    a, b = rand(rng, 9, n, np.uint32), rand(rng, 9, n, np.uint32)
    a[0], b[0] = 0xFFFFFFFF, 0
    b[0, 0] = 1
    got, carry = run_add(B, ctx, a, b)
    check(orc, a, b, got, carry)
    assert carry[0] == 1 and not got[0].any()


def test_carry_chain_at_every_boundary(B, ctx, orc):
    """A carry generated at limb k and propagated through all-ones limbs up to
    limb j, for k, j at lane, row and wave boundaries."""
    n = 512
    ks = [0, 1, 3, 4, 63, 64, 65, 127, 128, 255, 256, 300, 511]
    rows_a, rows_b = [], []
    for k in ks:
        for j in ks:
            if j < k:
                continue
            a = np.zeros(n, np.uint32)
            b = np.zeros(n, np.uint32)
            a[k] = 0x80000000
            b[k] = 0x80000000          # generate at k
            a[k + 1: j + 1] = 0xFFFFFFFF  # propagate through j
            rows_a.append(a)
            rows_b.append(b)
    a, b = np.stack(rows_a), np.stack(rows_b)
    for dt in (np.uint32, np.uint64):
        x, y = a.view(dt), b.view(dt)
        got, carry = run_add(B, ctx, x, y)
        check(orc, x, y, got, carry)


@pytest.mark.parametrize("which", ["a", "b"])
def test_in_place(B, ctx, orc, which):
    rng = np.random.default_rng(9)
    for n, dt in ((16, np.uint64), (300, np.uint32), (4096, np.uint64)):
        a, b = rand(rng, 33, n, dt), rand(rng, 33, n, dt)
        a[::2] = np.iinfo(dt).max
        got, carry = run_add(B, ctx, a, b, in_place=which)
        check(orc, a, b, got, carry)


def test_batch_one_and_without_carry(B, ctx, orc):
    rng = np.random.default_rng(4)
    a, b = rand(rng, 1, 40, np.uint32), rand(rng, 1, 40, np.uint32)
    A, Bt = G.to_dev(a), G.to_dev(b)
    out = G.empty_dev(a.shape, a.dtype)
    B.bigadd(ctx, A, Bt, out, None)
    G.sync()
    want, _ = orc.add(a, b)
    assert (G.from_dev(out, a.dtype) == want).all()


def test_ragged(B, ctx, orc):
    import torch
    rng = np.random.default_rng(12)
    for lb, dt in ((32, np.uint32), (64, np.uint64)):
        ns = np.array([1, 2, 3, 63, 64, 65, 129, 500, 4096 if lb == 64 else 8192, 7, 1000], dtype=np.int64)
        a_off = np.concatenate([[0], np.cumsum(ns)[:-1]]).astype(np.uint64)
        tot = int(ns.sum())
        # b holds the instances in reverse order
        bpos = np.concatenate([[0], np.cumsum(ns[::-1])[:-1]])[::-1].astype(np.uint64)
        A = rng.integers(0, np.iinfo(dt).max, tot, dtype=dt, endpoint=True)
        Bv = rng.integers(0, np.iinfo(dt).max, tot, dtype=dt, endpoint=True)
        A[: ns[0] + ns[1]] = np.iinfo(dt).max
        out_off = a_off + np.uint64(5)
        dev_out = G.empty_dev((tot + 5,), dt)
        carry = torch.zeros(len(ns), dtype=torch.uint8, device="cuda")
        desc = G.desc_dev(a_off, bpos, out_off, ns)
        B.bigadd_v(ctx, G.to_dev(A), G.to_dev(Bv), dev_out, carry, desc, len(ns), lb)
        G.sync()
        got = G.from_dev(dev_out, dt)
        cg = carry.cpu().numpy()
        pairs = [(A[int(a_off[i]): int(a_off[i]) + n].view(np.uint32), Bv[int(bpos[i]): int(bpos[i]) + n].view(np.uint32))
                 for i, n in enumerate(ns.tolist())]
        want = orc.add_ragged(pairs)
        for i, n in enumerate(ns.tolist()):
            oo = int(out_off[i])
            assert (got[oo: oo + n].view(np.uint32) == want[i][0]).all(), i
            assert cg[i] == want[i][1], i


@pytest.mark.parametrize("bits", W.ADD_SWEEP_BITS)
def test_full_sweep_size(B, ctx, orc, bits):
    """The benchmark's workload at full size (1 GiB of operands), every output
    limb and carry compared with the oracle."""
    a, b = W.add_sweep_inputs(bits)
    got, carry = run_add(B, ctx, a, b)
    check(orc, a, b, got, carry)


@pytest.mark.parametrize("tune", ["4,1,65536,7", "2,0,16384,0", "8,1,131072,7", "4,0,8192,3", "2,1,4096,5"])
def test_tuning_variants(B, orc, tune, monkeypatch):
    """Every schedule the tuner can select (rows in flight, non-temporal
    hints, grid cap, one-wave-per-instance vs workgroup-cooperative) gives the
    same bits.  BI_ADD_TUNE is read when a context is created."""
    monkeypatch.setenv("BI_ADD_TUNE", tune)
    c = B.Context(0)
    try:
        rng = np.random.default_rng(zlib.crc32(tune.encode()))
        for n, dt in ((1, np.uint32), (100, np.uint32), (128, np.uint64), (255, np.uint64), (256, np.uint64),
                      (300, np.uint64), (512, np.uint64), (1000, np.uint32), (2048, np.uint64), (4096, np.uint64)):
            a, b = rand(rng, 37, n, dt), rand(rng, 37, n, dt)
            a[::2] = np.iinfo(dt).max
            b[::4] = 0
            b[::4, 0] = 1
            got, carry = run_add(B, c, a, b)
            check(orc, a, b, got, carry)
    finally:
        c.close()
