"""Parity of bigmul_large (one product beyond 2^18 bits) with the CPU
oracle's schoolbook product, bit-exact.  The default path (AUTO, NTT) is a
two-dimensional NTT convolution over blocks of 2^14..2^18 bits; a forced
VALU, MFMA or PrimeField64 algorithm runs k^2 block products instead.  Sizes
around the block boundaries with ragged last blocks and around the 64-block
limit of the column transform, all-ones operands (every coefficient and carry
at its largest), u32 and u64 limbs, products of 2^21 and 2^22 bits in full,
and the 2^24-bit maximum (low words and residues)."""
from __future__ import annotations

import numpy as np
import pytest

from tests import gpu_util as G

pytestmark = pytest.mark.gpu

BLOCK = 8192


@pytest.fixture(scope="module")
def B():
    import paper_2405_14642_amd as B
    return B


@pytest.fixture(scope="module")
def ctx(B):
    c = B.Context(0)
    yield c
    c.close()


def run(B, ctx, a, b, algo=0, block_bits=0):
    A, Bt = G.to_dev(a), G.to_dev(b)
    out = G.empty_dev(2 * a.shape[0], a.dtype)
    B.bigmul_large(ctx, A, Bt, out, algo=algo, block_bits=block_bits)
    G.sync()
    return G.from_dev(out, a.dtype)


def check(orc, a, b, got):
    want = orc.mul(a[None, :], b[None, :])[0]
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"{bad.size} limbs differ, first at {bad[:8]}"


@pytest.mark.parametrize("n", [1, 5, BLOCK - 1, BLOCK, BLOCK + 1, 2 * BLOCK, 3 * BLOCK + 100, 4 * BLOCK - 7])
def test_sizes_uniform(B, ctx, orc, n):
    rng = np.random.default_rng(n + 11)
    a = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    b = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    check(orc, a, b, run(B, ctx, a, b))


@pytest.mark.parametrize("n", [BLOCK + 1, 3 * BLOCK + 100])
def test_all_ones(B, ctx, orc, n):
    a = np.full(n, 0xFFFFFFFF, dtype=np.uint32)
    check(orc, a, a.copy(), run(B, ctx, a, a.copy()))
    rng = np.random.default_rng(n)
    b = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    check(orc, a, b, run(B, ctx, a, b))


def test_u64_limbs(B, ctx, orc):
    n = BLOCK // 2 + 3  # 64-bit limbs: 8198 words, two blocks
    rng = np.random.default_rng(64)
    a = rng.integers(0, 2**64, n, dtype=np.uint64, endpoint=False)
    b = rng.integers(0, 2**64, n, dtype=np.uint64, endpoint=False)
    check(orc, a, b, run(B, ctx, a, b))


def test_2_21_bits(B, ctx, orc):
    n = 1 << 16  # 8 x 8 block products
    rng = np.random.default_rng(21)
    a = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    b = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    check(orc, a, b, run(B, ctx, a, b))


def test_repeat_after_smaller(B, ctx, orc):
    """Context scratch sized by a larger call serves a smaller one again."""
    rng = np.random.default_rng(3)
    for n in (5 * BLOCK + 1, BLOCK + 3):
        a = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
        b = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
        check(orc, a, b, run(B, ctx, a, b))


@pytest.mark.parametrize("algo", [1, 2, 3, 4, 5])
def test_block_algorithms(B, ctx, orc, algo):
    """Every algorithm (3: the NTT path; others: block products of that
    algorithm) gives the same product."""
    n = 2 * BLOCK + 3
    rng = np.random.default_rng(algo)
    a = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    b = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    check(orc, a, b, run(B, ctx, a, b, algo))


@pytest.mark.parametrize("algo", [0, 2])
@pytest.mark.parametrize("block_bits", [1 << 14, 1 << 15, 1 << 16, 1 << 17, 1 << 18])
@pytest.mark.parametrize("n", [1, 511, 513, 2047, 2049, 3 * 4096 + 5, 32768, 40000])
def test_block_sizes(B, ctx, orc, algo, block_bits, n):
    """Every block size of either path gives the same product, around its
    block boundaries (the NTT path takes at most 64 blocks, block products
    2^16..2^18-bit blocks)."""
    bw = block_bits // 32
    if (algo == 0 and -(-n // bw) > 64) or (algo == 2 and block_bits < (1 << 16)):
        pytest.skip("block size not taken by this path at this size")
    if n not in _ORACLE_CACHE:  # one oracle product per size, shared by every block size and path
        rng = np.random.default_rng(n)
        a = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
        b = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
        if n in (513, 2049):
            a[:] = 0xFFFFFFFF
            b[:] = 0xFFFFFFFF
        _ORACLE_CACHE[n] = (a, b, orc.mul(a[None, :], b[None, :])[0])
    a, b, want = _ORACLE_CACHE[n]
    got = run(B, ctx, a, b, algo, block_bits)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"{bad.size} limbs differ, first at {bad[:8]}"


_ORACLE_CACHE = {}


@pytest.mark.parametrize("n", [64 * 512 - 1, 64 * 512, 64 * 512 + 1, 64 * 1024 + 1, 5 * 8192 + 17])
def test_ntt_block_count_edges(B, ctx, orc, n):
    """Automatic blocks around the column transform's 64-block limit (the
    block size doubles past it) and at several column lengths."""
    rng = np.random.default_rng(n)
    a = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    b = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    a[-1] = b[-1] = 0xFFFFFFFF
    check(orc, a, b, run(B, ctx, a, b))


@pytest.mark.parametrize("n", [1 << 17, 1 << 18, 1 << 19])
def test_large_all_ones(B, ctx, orc, n):
    """Products of 2^22, 2^23 and 2^24 bits of all-ones operands: (2^N - 1)^2,
    every entry of the two-dimensional convolution at its bound, checked in
    full against the closed form.  In the final addition of the low and high
    words the carry out of the lowest 2048-word tile runs through every tile
    of the lower half (63, 127 and 255 tiles that only propagate), and so
    does the upper half's from the middle tile."""
    a = np.full(n, 0xFFFFFFFF, dtype=np.uint32)
    got = run(B, ctx, a, a.copy())
    exp = np.concatenate([[1], np.zeros(n - 1), [0xFFFFFFFE], np.full(n - 1, 0xFFFFFFFF)]).astype(np.uint32)
    assert (got == exp).all()


def test_2_22_bits(B, ctx, orc):
    n = 1 << 17
    rng = np.random.default_rng(22)
    a = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    b = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    check(orc, a, b, run(B, ctx, a, b))


def _mod(x: np.ndarray, p: int) -> int:
    """Value of a little-endian u32 limb array mod p (Horner, high limb first)."""
    r = 0
    for v in x[::-1].tolist():
        r = (r * (1 << 32) + v) % p
    return r


def test_max_size_sampled(B, ctx, orc):
    """2^24-bit operands (the largest size, 64 blocks of 2^18 bits): the lowest
    8192 words equal the oracle's product of the operands' lowest 8192 words
    (they depend on nothing else), and the whole product agrees with a * b
    modulo three 61-bit primes."""
    n = (1 << 24) // 32
    rng = np.random.default_rng(24)
    a = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    b = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    got = run(B, ctx, a, b)
    low = orc.mul(a[None, :BLOCK], b[None, :BLOCK])[0][:BLOCK]
    assert (got[:BLOCK] == low).all()
    for p in ((1 << 61) - 1, (1 << 61) - 31, 2305843009213693921):
        assert _mod(got, p) == _mod(a, p) * _mod(b, p) % p, p
