"""Host-side pins of the NTT prime-field set-up (Section 4.1), no GPU needed."""
from __future__ import annotations

import json
import os

import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "prime_fields.json")
LIB_PRIMES = (2113929217, 2130706433)  # the two primes the NTT path uses


@pytest.fixture(scope="module")
def B():
    import paper_2405_14642_amd as B
    return B


def trial_division_prime(n: int) -> bool:
    if n < 2:
        return False
    f = 2
    while f * f <= n:
        if n % f == 0:
            return False
        f += 1 if f == 2 else 2
    return True


def test_paper_fields_golden(B):
    """The paper's printed fields: p = k 2^n + 1 is prime and the printed g is a
    2^n-th root of unity of exact order 2^n; the library's search on the same p
    returns the same k and n and a root of the same exact order."""
    fields = json.load(open(GOLDEN))["fields"]
    for f in fields:
        p, k, n, g = f["p"], f["k"], f["n"], f["g"]
        assert p == k * (1 << n) + 1
        assert pow(g, 1 << n, p) == 1 and pow(g, 1 << (n - 1), p) == p - 1
        if p < (1 << 40):
            assert trial_division_prime(p)
        info = B.ntt_field(p)
        assert (info.p, info.k, info.two_adicity) == (p, k, n)
        assert pow(info.g, 1 << n, p) == 1 and pow(info.g, 1 << (n - 1), p) == p - 1
        assert info.g == pow(info.a, k, p)
        # the search takes the first a: every smaller a gives a root of lower order
        for a in range(2, info.a):
            assert pow(pow(a, k, p), 1 << (n - 1), p) == 1


@pytest.mark.parametrize("p", LIB_PRIMES)
def test_library_primes(B, p):
    assert p < (1 << 31) and trial_division_prime(p)
    info = B.ntt_field(p)
    assert info.two_adicity >= 15 and p == info.k * (1 << info.two_adicity) + 1
    assert pow(info.g, 1 << (info.two_adicity - 1), p) == p - 1


def test_crt_bound():
    """Every coefficient of a product of two 2^18-bit integers in 16-bit digits
    is below 2^14 (2^16 - 1)^2 < p1 p2, so CRT recovers it exactly."""
    n16 = (1 << 18) // 16
    assert n16 * (2 ** 16 - 1) ** 2 < LIB_PRIMES[0] * LIB_PRIMES[1]


@pytest.mark.parametrize("bad", [0, 1, 2, 4, 9, 3221225471, (1 << 63) + 1])
def test_rejects_non_primes(B, bad):
    with pytest.raises(B.BigIntError):
        B.ntt_field(bad)


PF64 = 4179340454199820289  # PrimeField64 of Section 4.1, the BI_MUL_NTT_PF64 modulus


def test_pf64_single_prime_bound():
    """One PrimeField64 residue determines every coefficient: 16-bit digits of
    2^18-bit operands give coefficients below 2^14 (2^16 - 1)^2 < 2^46 < p, and
    the half-length split needs (cyc +- neg) < 2p as well."""
    fields = {f["name"]: f for f in json.load(open(GOLDEN))["fields"]}
    assert fields["PrimeField64"]["p"] == PF64
    bound = ((1 << 18) // 16) * (2 ** 16 - 1) ** 2
    assert bound < 2 ** 46 and 2 * bound < PF64


def test_pf64_montgomery_constants():
    """p = 1 + 29 2^57, so -p^-1 mod 2^64 = 29 2^57 - 1 and m p = m + 29 m 2^57:
    the shift forms the 64-bit Montgomery reduction uses."""
    assert PF64 == 29 * (1 << 57) + 1
    pinv_neg = (29 << 57) - 1
    assert (PF64 * pinv_neg) % (1 << 64) == (1 << 64) - 1
    assert pinv_neg == (-pow(PF64, -1, 1 << 64)) % (1 << 64)
    # two-adicity 57 leaves room for the twist root of order 2^15
    assert (PF64 - 1) % (1 << 15) == 0


def test_negacyclic_split_identity():
    """c = a b, c = c_lo + x^H c_hi: the cyclic convolution of length H gives
    c_lo + c_hi and the negacyclic one c_lo - c_hi, so their half-sum and
    half-difference are c_lo and c_hi (checked on integer vectors)."""
    import random
    rng = random.Random(5)
    for H in (1, 2, 4, 8, 16):
        a = [rng.randrange(1 << 16) for _ in range(H)]
        b = [rng.randrange(1 << 16) for _ in range(H)]
        c = [0] * (2 * H)
        for i in range(H):
            for j in range(H):
                c[i + j] += a[i] * b[j]
        cyc = [0] * H
        neg = [0] * H
        for i in range(H):
            for j in range(H):
                k = i + j
                cyc[k % H] += a[i] * b[j]
                neg[k % H] += a[i] * b[j] * (1 if k < H else -1)
        assert [(x + y) // 2 for x, y in zip(cyc, neg)] == c[:H]
        assert [(x - y) // 2 for x, y in zip(cyc, neg)] == c[H:]
