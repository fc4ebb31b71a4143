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
