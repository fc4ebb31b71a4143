"""Checks that pin the CPU oracle to things other than itself.

Each check takes a bound oracle (the real one, or a copy of its C source with
a planted mistake) and raises AssertionError on a mismatch.  The sources of
truth are: Python's own bignum arithmetic (an independent library routine),
closed forms of the results, and algebraic invariants.
"""
from __future__ import annotations

import itertools

import numpy as np

import oracle as O

SPECIAL32 = (0, 1, 2, 0x7FFFFFFF, 0x80000000, 0xFFFFFFFE, 0xFFFFFFFF)


def _ints(x):
    return [O.to_int(r) for r in np.atleast_2d(x)]


def check_add_bruteforce(orc, nmax=3):
    """Every combination of special limb values for n <= 2, plus random n <= nmax,
    against Python integer addition."""
    rng = np.random.default_rng(1)
    for n in range(1, nmax + 1):
        if n <= 2:
            combos = np.array(list(itertools.product(SPECIAL32, repeat=2 * n)), dtype=np.uint32)
        else:
            combos = rng.choice(np.array(SPECIAL32, dtype=np.uint32), size=(4000, 2 * n))
        combos = np.concatenate([combos, rng.integers(0, 1 << 32, size=(500, 2 * n), dtype=np.uint64).astype(np.uint32)])
        a, b = combos[:, :n].copy(), combos[:, n:].copy()
        out, carry = orc.add(a, b)
        for i in range(a.shape[0]):
            s = O.to_int(a[i]) + O.to_int(b[i])
            assert O.to_int(out[i]) == s % (1 << (32 * n)), (n, i)
            assert int(carry[i]) == s >> (32 * n), (n, i)


def check_mul_bruteforce(orc, nmax=3):
    rng = np.random.default_rng(2)
    for n in range(1, nmax + 1):
        if n <= 2:
            combos = np.array(list(itertools.product(SPECIAL32, repeat=2 * n)), dtype=np.uint32)
        else:
            combos = rng.choice(np.array(SPECIAL32, dtype=np.uint32), size=(4000, 2 * n))
        combos = np.concatenate([combos, rng.integers(0, 1 << 32, size=(500, 2 * n), dtype=np.uint64).astype(np.uint32)])
        a, b = combos[:, :n].copy(), combos[:, n:].copy()
        out = orc.mul(a, b)
        for i in range(a.shape[0]):
            assert O.to_int(out[i]) == O.to_int(a[i]) * O.to_int(b[i]), (n, i)


def check_against_python(orc, a, b, do_mul=True):
    """Sampled pairs of a workload against Python's bignum."""
    out, carry = orc.add(a, b)
    w = a.dtype.itemsize * 8
    n = a.shape[1]
    for i in range(a.shape[0]):
        s = O.to_int(a[i]) + O.to_int(b[i])
        assert O.to_int(out[i]) == s % (1 << (w * n))
        assert int(carry[i]) == s >> (w * n)
    if do_mul:
        prod = orc.mul(a, b)
        for i in range(a.shape[0]):
            assert O.to_int(prod[i]) == O.to_int(a[i]) * O.to_int(b[i])


def check_closed_forms(orc, sizes=(1, 2, 3, 7, 64, 129)):
    M = 0xFFFFFFFF
    for n in sizes:
        ones = np.full((1, n), M, dtype=np.uint32)
        one = np.zeros((1, n), dtype=np.uint32)
        one[0, 0] = 1
        # Section 2: the carry of the lowest limb runs through every limb.
        out, carry = orc.add(ones, one)
        assert not out.any() and carry[0] == 1
        out, carry = orc.add(one, ones)
        assert not out.any() and carry[0] == 1
        # all-ones + all-ones = 2^(N+1) - 2: limb0 = 2^32 - 2, others all-ones, carry 1.
        out, carry = orc.add(ones, ones)
        assert out[0, 0] == M - 1 and (out[0, 1:] == M).all() and carry[0] == 1
        # (2^N - 1)^2 = 2^(2N) - 2^(N+1) + 1: limbs [1, 0 x (n-1), 2^32-2, (2^32-1) x (n-1)]
        sq = orc.mul(ones, ones)[0]
        exp = np.concatenate([[1], np.zeros(n - 1), [M - 1], np.full(n - 1, M)]).astype(np.uint32)
        assert (sq == exp).all(), n
        # a * 1 = a, a * 0 = 0, a + 0 = a
        rng = np.random.default_rng(n)
        a = rng.integers(0, 1 << 32, size=(1, n), dtype=np.uint64).astype(np.uint32)
        p = orc.mul(a, one)[0]
        assert (p[:n] == a[0]).all() and not p[n:].any()
        assert not orc.mul(a, np.zeros_like(a)).any()
        s, c = orc.add(a, np.zeros_like(a))
        assert (s == a).all() and c[0] == 0
    # 2^i * 2^j = 2^(i+j), all i, j < 32 n for n = 3
    n = 3
    bits = 32 * n
    e = np.zeros((bits, n), dtype=np.uint32)
    for i in range(bits):
        e[i, i // 32] = np.uint32(1 << (i % 32))
    A = np.repeat(e, bits, axis=0)
    B = np.tile(e, (bits, 1))
    P = orc.mul(A, B)
    for i in range(bits):
        for j in range(bits):
            v = P[i * bits + j]
            k = i + j
            want = np.zeros(2 * n, dtype=np.uint32)
            want[k // 32] = np.uint32(1 << (k % 32))
            assert (v == want).all(), (i, j)


def _residue(x: np.ndarray, p: int) -> np.ndarray:
    """Residues mod p (< 2^20) of each row of little-endian u32 limbs, by Horner
    from the top limb: r = (r * 2^32 + limb) mod p."""
    x = np.atleast_2d(x).astype(np.uint64)
    r = np.zeros(x.shape[0], dtype=np.uint64)
    base = np.uint64((1 << 32) % p)
    P = np.uint64(p)
    for k in range(x.shape[1] - 1, -1, -1):
        r = (r * base + x[:, k] % P) % P
    return r


def check_invariants(orc, n=40, batch=64, seed=7):
    rng = np.random.default_rng(seed)
    a = rng.integers(0, 1 << 32, size=(batch, n), dtype=np.uint64).astype(np.uint32)
    b = rng.integers(0, 1 << 32, size=(batch, n), dtype=np.uint64).astype(np.uint32)
    a[: batch // 4] = 0xFFFFFFFF  # carry-heavy quarter
    # commutativity
    s1, c1 = orc.add(a, b)
    s2, c2 = orc.add(b, a)
    assert (s1 == s2).all() and (c1 == c2).all()
    assert (orc.mul(a, b) == orc.mul(b, a)).all()
    # (a + b) - b == a, checked as (a + b) + (2^N - b) == a + 2^N
    nb = (~b).astype(np.uint32)
    one = np.zeros_like(b)
    one[:, 0] = 1
    negb, _ = orc.add(nb, one)  # 2^N - b (mod 2^N)
    back, _ = orc.add(s1, negb)
    assert (back == a).all()
    # residues modulo small primes and modulo 2^32 - 1 / 2^32 + 1
    prod = orc.mul(a, b)
    sum_full = np.concatenate([s1, c1[:, None].astype(np.uint32)], axis=1)
    for p in (3, 5, 7, 65521, 1000003):
        ra, rb = _residue(a, p), _residue(b, p)
        P = np.uint64(p)
        assert (_residue(prod, p) == (ra * rb) % P).all(), p
        assert (_residue(sum_full, p) == (ra + rb) % P).all(), p
    m1 = (1 << 32) - 1  # 2^32 = 1 mod m1: residue = sum of limbs
    m2 = (1 << 32) + 1  # 2^32 = -1 mod m2: alternating sum

    def r1(x):
        return [sum(int(v) for v in row) % m1 for row in np.atleast_2d(x)]

    def r2(x):
        return [sum(int(v) * (1 if k % 2 == 0 else -1) for k, v in enumerate(row)) % m2 for row in np.atleast_2d(x)]

    for f, m in ((r1, m1), (r2, m2)):
        for x, y, z in zip(f(a), f(b), f(prod)):
            assert z == (x * y) % m
    # (a + b)^2 == a^2 + 2ab + b^2, with one zero limb of headroom
    z = np.zeros((batch, 1), dtype=np.uint32)
    A, B = np.concatenate([a, z], 1), np.concatenate([b, z], 1)
    S, cs = orc.add(A, B)
    assert not cs.any()
    lhs = orc.mul(S, S)
    aa, bb, ab = orc.mul(A, A), orc.mul(B, B), orc.mul(A, B)
    ab2, c0 = orc.add(ab, ab)
    t, c1_ = orc.add(aa, ab2)
    rhs, c2_ = orc.add(t, bb)
    assert not (c0.any() or c1_.any() or c2_.any())
    assert (lhs == rhs).all()


def check_u64_view(orc):
    """u64 limbs give the same bytes as the u32 view with twice the limbs."""
    rng = np.random.default_rng(11)
    a = rng.integers(0, 1 << 63, size=(8, 5), dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    b = rng.integers(0, 1 << 63, size=(8, 5), dtype=np.uint64)
    a[0] = np.uint64(0xFFFFFFFFFFFFFFFF)
    b[0] = 0
    b[0, 0] = 1
    out, carry = orc.add(a, b)
    for i in range(8):
        s = O.to_int(a[i]) + O.to_int(b[i])
        assert O.to_int(out[i]) == s % (1 << 320) and carry[i] == s >> 320
    prod = orc.mul(a, b)
    assert prod.dtype == np.uint64 and prod.shape == (8, 10)
    for i in range(8):
        assert O.to_int(prod[i]) == O.to_int(a[i]) * O.to_int(b[i])


def check_ragged(orc):
    rng = np.random.default_rng(5)
    pairs = []
    for n in (1, 2, 5, 33, 100):
        pairs.append((rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32),
                      rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)))
    outs = orc.mul_ragged(pairs)
    for (x, y), o in zip(pairs, outs):
        assert O.to_int(o) == O.to_int(x) * O.to_int(y)
    # ragged sums, with an all-ones + 1 pair (the carry crosses every limb)
    # and an all-ones + all-ones pair among them
    pairs.append((np.full(7, 0xFFFFFFFF, np.uint32), np.array([1, 0, 0, 0, 0, 0, 0], np.uint32)))
    pairs.append((np.full(3, 0xFFFFFFFF, np.uint32), np.full(3, 0xFFFFFFFF, np.uint32)))
    sums = orc.add_ragged(pairs)
    for (x, y), (o, c) in zip(pairs, sums):
        n = len(x)
        s = O.to_int(x) + O.to_int(y)
        assert len(o) == n and O.to_int(o) == s % (1 << (32 * n)) and c == s >> (32 * n)
    assert sums[-2][1] == 1 and not sums[-2][0].any()


ALL_FAST = (check_add_bruteforce, check_mul_bruteforce, check_closed_forms, check_invariants,
            check_u64_view, check_ragged)
