"""Fused programs of Section 6.1 (bi_fused): 6-Add and Poly in one workgroup
per instance, bit-exact against the oracle's compositions of add and the
same-length product."""
from __future__ import annotations

import numpy as np
import pytest

import oracle as O
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

PROGRAMS = {"add6": 1, "poly": 2, "mullow": 3}


@pytest.fixture(scope="module")
def B():
    import paper_2405_14642_amd as B
    return B


@pytest.fixture(scope="module")
def ctx(B):
    c = B.Context(0)
    yield c
    c.close()


def want(orc, name, a, b):
    return {"add6": O.add6, "poly": O.poly, "mullow": O.mul_low}[name](a, b)


def run(B, ctx, prog, a, b):
    A, Bt = G.to_dev(a), G.to_dev(b)
    out = G.empty_dev(a.shape, a.dtype)
    B.fused(ctx, prog, A, Bt, out)
    G.sync()
    return G.from_dev(out, a.dtype)


def operands(rng, batch, n, dt=np.uint32):
    info = np.iinfo(dt)
    a = rng.integers(0, info.max, (batch, n), dtype=dt, endpoint=True)
    b = rng.integers(0, info.max, (batch, n), dtype=dt, endpoint=True)
    a[0] = b[0] = info.max                       # every carry chain runs the full length
    if batch > 1:
        a[1] = info.max
        b[1] = 0
        b[1, 0] = 1                               # all-ones + 1 wraps to 0
    if batch > 2:
        a[2] = 0                                  # zero operand
    if batch > 3:
        a[3] = info.max // 255 * 0x80
        b[3] = info.max // 255 * 0x7F
    return a, b


SIZES = [1, 2, 3, 4, 5, 7, 8, 31, 32, 33, 63, 64, 65, 100, 127, 128, 129, 255, 256, 257, 511, 512, 513, 1000,
         1023, 1024, 1025, 2047, 2048, 2049, 4095, 4096, 4097, 8191, 8192]


@pytest.mark.parametrize("name", list(PROGRAMS))
@pytest.mark.parametrize("n", SIZES)
def test_sizes(B, ctx, orc, name, n):
    rng = np.random.default_rng(n)
    batch = 6 if n <= 1024 else 3
    a, b = operands(rng, batch, n)
    got = run(B, ctx, PROGRAMS[name], a, b)
    exp = want(orc, name, a, b)
    bad = np.nonzero((got != exp).any(axis=1))[0]
    assert bad.size == 0, f"{name} n={n}: rows {bad.tolist()} differ"


@pytest.mark.parametrize("name", ["poly", "mullow"])
@pytest.mark.parametrize("n", [1, 2, 5, 16, 17, 31, 32, 33, 64, 65, 96, 128, 130, 200, 255, 256])
def test_packed_many_instances(B, ctx, orc, name, n):
    """Instances of up to 256 words run several per wavefront: batches of
    many wavefronts with a partial last one, every instance checked."""
    rng = np.random.default_rng(500 + n)
    batch = 333
    a, b = operands(rng, batch, n)
    got = run(B, ctx, PROGRAMS[name], a, b)
    exp = want(orc, name, a, b)
    bad = np.nonzero((got != exp).any(axis=1))[0]
    assert bad.size == 0, f"{name} n={n}: rows {bad[:8].tolist()} differ"


@pytest.mark.parametrize("name", list(PROGRAMS))
def test_u64_limbs(B, ctx, orc, name):
    rng = np.random.default_rng(64)
    for n in (1, 3, 64, 513, 4096):
        a, b = operands(rng, 4, n, np.uint64)
        got = run(B, ctx, PROGRAMS[name], a, b)
        assert (got == want(orc, name, a, b)).all(), (name, n)


# Oracle work per (program, size) of the paper's batches, in u32 multiply-
# accumulates: every instance is checked while the whole batch fits it.
ORACLE_MAC_BUDGET = 1 << 36


@pytest.mark.parametrize("name", list(PROGRAMS))
@pytest.mark.parametrize("bits", [1 << 10, 1 << 12, 1 << 15, 1 << 18])
def test_paper_workload(B, ctx, orc, name, bits):
    """NumBits x NumInsts = 2^32 (the paper's batches, u64 limbs), one launch
    over the whole batch.  6-Add: every instance against the oracle.  The
    products: every instance while the oracle's schoolbook work (n^2 u32
    multiply-accumulates per product, four products per Poly) stays within
    ORACLE_MAC_BUDGET, which covers every size up to 2^12 bits; above it an
    evenly strided subset of that cost plus the first four rows (the edge
    patterns) and the last."""
    n = bits // 64
    batch = (1 << 32) // bits
    rng = np.random.default_rng(bits)
    a, b = operands(rng, batch, n, np.uint64)
    got = run(B, ctx, PROGRAMS[name], a, b)
    per_inst = {"add6": 0, "mullow": 1, "poly": 4}[name] * (2 * n) ** 2
    if per_inst * batch <= ORACLE_MAC_BUDGET:
        pick = np.arange(batch)
    else:
        cnt = ORACLE_MAC_BUDGET // per_inst
        pick = np.unique(np.concatenate([np.arange(4), np.linspace(0, batch - 1, cnt).astype(np.int64)]))
    exp = want(orc, name, a[pick], b[pick])
    bad = np.nonzero((got[pick] != exp).any(axis=1))[0]
    assert bad.size == 0, f"{name} at {bits} bits: {bad.size} of {pick.size} checked instances differ, " \
                          f"first {pick[bad[:8]].tolist()}"
