"""Parity of bigadd_large (one integer carried across workgroups) with the
CPU oracle's addition, bit-exact: sizes around the chunk, row and tile
boundaries with ragged tails, every chunk width (pointer alignment), u32 and
u64 limbs, in-place, carry patterns that cross tile boundaries, and the
2^32-bit workload in full."""
from __future__ import annotations

import numpy as np
import pytest

import workloads as W
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

TILE = 4096  # 32-bit words per tile at 16-byte chunks (1024 chunks)


@pytest.fixture(scope="module")
def B():
    import paper_2405_14642_amd as B
    return B


@pytest.fixture(scope="module")
def ctx(B):
    c = B.Context(0)
    yield c
    c.close()


def run(B, ctx, a, b, shift=0, in_place=None, carry=True):
    """bigadd_large on device copies of a and b placed `shift` limbs into
    their buffers (shift changes the chunk width the pointers allow)."""
    import torch
    n = a.shape[0]
    A = G.to_dev(np.concatenate([np.zeros(shift, a.dtype), a]))[shift:]
    Bt = G.to_dev(np.concatenate([np.zeros(shift, b.dtype), b]))[shift:]
    if in_place == "a":
        out = A
    elif in_place == "b":
        out = Bt
    else:
        out = G.empty_dev(n + shift, a.dtype)[shift:]
    c = torch.full((1,), 7, dtype=torch.uint8, device="cuda") if carry else None
    B.bigadd_large(ctx, A, Bt, out, c)
    G.sync()
    return G.from_dev(out, a.dtype), (int(c.item()) if carry else None)


def check(orc, a, b, got, carry):
    want, wc = orc.add(a[None, :], b[None, :])
    bad = np.nonzero(got != want[0])[0]
    assert bad.size == 0, f"{bad.size} limbs differ, first at {bad[:8]}"
    if carry is not None:
        assert carry == int(wc[0])


def tile_patterns(rng, n, dt):
    """a uniform; b = ~a (every limb propagates) except: whole tiles left
    propagating, tiles that generate at their top limb, tiles with a kill
    in the middle, so tile carry-ins arrive through runs of all-ones tiles."""
    a = rng.integers(0, np.iinfo(dt).max, size=n, dtype=dt, endpoint=True)
    b = ~a
    per_tile = TILE * 4 // np.dtype(dt).itemsize
    for t in range((n + per_tile - 1) // per_tile):
        lo, hi = t * per_tile, min(n, (t + 1) * per_tile)
        kind = rng.integers(0, 4)
        if kind == 1:  # generate at the top limb of the tile
            a[hi - 1] = np.iinfo(dt).max
            b[hi - 1] = 1
        elif kind == 2:  # kill then generate in the middle
            j = int(rng.integers(lo, hi))
            a[j], b[j] = 0, 0
            if j + 1 < hi:
                a[j + 1], b[j + 1] = np.iinfo(dt).max, 2
    a[0], b[0] = np.iinfo(dt).max, 1  # a carry enters at limb 0
    return a, b


SIZES = [1, 2, 3, 4, 5, 63, 64, 65, 255, 256, 257, 1023, 1024, 1025, TILE - 1, TILE, TILE + 1,
         3 * TILE + 17, 8 * TILE - 3, 65536 + 7, (1 << 20) + 13]


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("shift", [0, 1, 2])
def test_sizes_widths_uniform(B, ctx, orc, n, shift):
    rng = np.random.default_rng(1000 + n * 3 + shift)
    a = rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)
    b = rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)
    got, c = run(B, ctx, a, b, shift)
    check(orc, a, b, got, c)


@pytest.mark.parametrize("n", [1, 65, TILE + 1, 5 * TILE + 9, (1 << 20) + 13])
@pytest.mark.parametrize("shift", [0, 1, 2])
def test_ripple(B, ctx, orc, n, shift):
    a, b = W.large_add_inputs(n, "ripple")
    got, c = run(B, ctx, a, b, shift)
    assert c == 1 and not got.any()
    check(orc, a, b, got, c)


@pytest.mark.parametrize("n", [TILE * 9 + 5, (1 << 20) + 13, 1 << 22])
@pytest.mark.parametrize("shift", [0, 1, 2])
def test_tile_carry_patterns(B, ctx, orc, n, shift):
    rng = np.random.default_rng(n + shift)
    a, b = tile_patterns(rng, n, np.uint32)
    got, c = run(B, ctx, a, b, shift)
    check(orc, a, b, got, c)


@pytest.mark.parametrize("n", [TILE * 3 + 1, 1 << 22])
def test_chains_and_all_ones(B, ctx, orc, n):
    a, b = W.large_add_inputs(n, "chains")
    got, c = run(B, ctx, a, b)
    check(orc, a, b, got, c)
    b2 = ~a  # the sum is all ones: no carry anywhere
    got, c = run(B, ctx, a, b2)
    assert c == 0 and (got == np.uint32(0xFFFFFFFF)).all()


@pytest.mark.parametrize("n", [1, 3, TILE // 2 + 1, (1 << 19) + 5])
@pytest.mark.parametrize("shift", [0, 1])
def test_u64(B, ctx, orc, n, shift):
    rng = np.random.default_rng(77 + n + shift)
    a, b = tile_patterns(rng, n, np.uint64)
    got, c = run(B, ctx, a, b, shift)
    check(orc, a, b, got, c)


@pytest.mark.parametrize("where", ["a", "b"])
def test_in_place_and_no_carry(B, ctx, orc, where):
    n = 3 * TILE + 11
    rng = np.random.default_rng(5)
    a, b = tile_patterns(rng, n, np.uint32)
    got, c = run(B, ctx, a, b, in_place=where)
    check(orc, a, b, got, c)
    got, c = run(B, ctx, a, b, carry=False)
    check(orc, a, b, got, None)


def test_workload_2_32_bits(B, ctx, orc):
    """The add sweep's 2^32 bits as one integer (2^27 u32 limbs), in full."""
    n = (1 << 32) // 32
    a, b = W.large_add_inputs(n)
    got, c = run(B, ctx, a, b)
    check(orc, a, b, got, c)
    a, b = W.large_add_inputs(n, "chains")
    got, c = run(B, ctx, a, b)
    check(orc, a, b, got, c)


def test_many_tiles_scan_runs(B, ctx, orc):
    """65537 tiles of 4-byte chunks: every scan thread folds several 16-byte
    summary words (the four-word loads and the remainder), and the summary
    padding is partial."""
    n = (1 << 26) + 3
    a, b = W.large_add_inputs(n, "chains")
    got, c = run(B, ctx, a, b, shift=1)
    check(orc, a, b, got, c)
