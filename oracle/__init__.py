"""CPU oracle for batched big-integer addition and multiplication.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only code that may import this package.  It shares no
code with the HIP library (``paper_2405_14642_amd``) and neither imports the
other; the seeded input generator in ``workloads`` is the only module both use.

What it computes (plain definitions, Section 2 and eq. (1) of Section 3.1):

* ``add(a, b)``  -> ((a + b) mod 2^(n w), carry out), limb by limb with a
  double-width sum; the carry out is the extra result the library returns
  beside the paper's same-length sum.
* ``mul(a, b)``  -> the full 2n-limb product a * b (schoolbook rows); the
  paper's same-length product is its low n limbs.
* ``add_ragged`` / ``mul_ragged`` -> the same per pair over a list of pairs
  of different lengths (one C call, pairs in parallel).
* ``mul_low(a, b)`` -> the paper's same-length product (Figs. 4-5): the low
  n limbs of ``mul``.
* ``add6(a, b)`` and ``poly(a, b)`` -> the fused programs of Section 6.1 in
  same-length arithmetic (mod 2^(n w)), composed from ``add`` and the low n
  limbs of ``mul`` in the order the program states: six additions in a chain
  (a + b, then + a, + b, + a, + b, + a), and (a a + b)(b b + b) + a b.

Arrays are numpy (batch, n) of uint32 or uint64 limbs, little-endian,
instance-major.  uint64 limbs are processed as twice as many uint32 limbs,
which is the same byte string on a little-endian host.

Pins (tests/test_oracle_pins.py): brute force against Python integers on all
small limb combinations, Python's own bignum at every workload size, closed
forms (all-ones + 1, (2^N - 1)^2, 2^i * 2^j), invariants (commutativity,
(a+b)^2 = a^2 + 2ab + b^2, residues modulo small primes and 2^32 +- 1), and
planted mistakes in a copy of the C source that the pins must catch.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(_HERE, "bigint_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def compile_source(src: str, out: str) -> str:
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", src, "-o", tmp])
    os.replace(tmp, out)
    return out


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(SOURCE):
        compile_source(SOURCE, _LIB)
    return _LIB


def _bind(path: str):
    lib = ctypes.CDLL(path)
    P, U64, I = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int
    lib.oracle_add.argtypes = [P, P, P, P, U64, U64, I]
    lib.oracle_mul.argtypes = [P, P, P, U64, U64, I]
    lib.oracle_mul_ragged.argtypes = [P, P, P, P, P, P, P, U64, I]
    lib.oracle_add_ragged.argtypes = [P, P, P, P, P, P, P, P, U64, I]
    for f in (lib.oracle_add, lib.oracle_mul, lib.oracle_mul_ragged, lib.oracle_add_ragged):
        f.restype = I
    return lib


class Oracle:
    """Bound oracle library (a planted-mistake copy can be bound the same way)."""

    def __init__(self, path: str):
        self.lib = _bind(path)
        self.last_threads = 0

    @staticmethod
    def _u32(x: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x)
        if x.dtype not in (np.uint32, np.uint64):
            raise TypeError("limbs must be uint32 or uint64")
        if x.ndim == 1:
            x = x[None, :]
        return x.view(np.uint32)

    def add(self, a: np.ndarray, b: np.ndarray, threads: int = 0):
        dtype = np.asarray(a).dtype
        a32, b32 = self._u32(a), self._u32(b)
        if a32.shape != b32.shape:
            raise ValueError("operand shapes differ")
        batch, n = a32.shape
        out = np.empty_like(a32)
        carry = np.empty(batch, dtype=np.uint8)
        self.last_threads = self.lib.oracle_add(a32.ctypes.data, b32.ctypes.data, out.ctypes.data,
                                                carry.ctypes.data, n, batch, threads)
        return out.view(dtype).reshape(batch, -1), carry

    def mul(self, a: np.ndarray, b: np.ndarray, threads: int = 0):
        dtype = np.asarray(a).dtype
        a32, b32 = self._u32(a), self._u32(b)
        if a32.shape != b32.shape:
            raise ValueError("operand shapes differ")
        batch, n = a32.shape
        out = np.empty((batch, 2 * n), dtype=np.uint32)
        self.last_threads = self.lib.oracle_mul(a32.ctypes.data, b32.ctypes.data, out.ctypes.data,
                                                n, batch, threads)
        return out.view(dtype).reshape(batch, -1)

    @staticmethod
    def _ragged_layout(pairs, out_per_limb):
        """Concatenated operands of a list of pairs: a in pair order, b in
        reverse pair order, results with one spare limb between pairs (so
        the three offset arrays all differ)."""
        ns = np.array([len(p[0]) for p in pairs], dtype=np.uint32)
        cnt = len(pairs)
        n64 = ns.astype(np.uint64)
        a_off = np.zeros(cnt, dtype=np.uint64)
        b_off = np.zeros(cnt, dtype=np.uint64)
        o_off = np.zeros(cnt, dtype=np.uint64)
        if cnt > 1:
            a_off[1:] = np.cumsum(n64[:-1])
            b_off[:-1] = np.cumsum(n64[::-1])[::-1][1:]
            o_off[1:] = np.cumsum(out_per_limb * n64[:-1] + 1)
        A = np.zeros(int(n64.sum()), np.uint32)
        B = np.zeros(int(n64.sum()), np.uint32)
        for p, (x, y) in enumerate(pairs):
            A[int(a_off[p]): int(a_off[p]) + int(ns[p])] = np.asarray(x, dtype=np.uint32)
            B[int(b_off[p]): int(b_off[p]) + int(ns[p])] = np.asarray(y, dtype=np.uint32)
        total_out = int(o_off[-1]) + out_per_limb * int(ns[-1]) + 1 if cnt else 0
        return ns, A, B, a_off, b_off, o_off, np.zeros(total_out, np.uint32)

    def mul_ragged(self, pairs, threads: int = 0):
        """pairs: list of (a, b) uint32 1-D arrays of equal length per pair;
        returns the list of 2n-limb products."""
        ns, A, B, ao, bo, oo, out = self._ragged_layout(pairs, 2)
        self.last_threads = self.lib.oracle_mul_ragged(A.ctypes.data, B.ctypes.data, out.ctypes.data,
                                                       ao.ctypes.data, bo.ctypes.data, oo.ctypes.data,
                                                       ns.ctypes.data, len(pairs), threads)
        return [out[int(o):int(o) + 2 * int(k)] for o, k in zip(oo, ns)]

    def add_ragged(self, pairs, threads: int = 0):
        """pairs: list of (a, b) uint32 1-D arrays of equal length per pair;
        returns the list of (sum mod 2^(32 n), carry out) per pair."""
        ns, A, B, ao, bo, oo, out = self._ragged_layout(pairs, 1)
        carry = np.empty(len(pairs), dtype=np.uint8)
        self.last_threads = self.lib.oracle_add_ragged(A.ctypes.data, B.ctypes.data, out.ctypes.data,
                                                       carry.ctypes.data, ao.ctypes.data, bo.ctypes.data,
                                                       oo.ctypes.data, ns.ctypes.data, len(pairs), threads)
        return [(out[int(o):int(o) + int(k)], int(c)) for o, k, c in zip(oo, ns, carry)]


_default: Oracle | None = None


def get() -> Oracle:
    global _default
    if _default is None:
        if not os.path.exists(_LIB):
            build()
        _default = Oracle(_LIB)
    return _default


def add(a, b, threads: int = 0):
    return get().add(a, b, threads)


def mul(a, b, threads: int = 0):
    return get().mul(a, b, threads)


def mul_ragged(pairs, threads: int = 0):
    return get().mul_ragged(pairs, threads)


def add_ragged(pairs, threads: int = 0):
    return get().add_ragged(pairs, threads)


def mul_low(a, b, threads: int = 0):
    """Same-length product: the low n limbs of the full product."""
    return np.ascontiguousarray(get().mul(a, b, threads)[:, : a.shape[1]])


_mul_low = mul_low


def add6(a, b, threads: int = 0):
    """Six additions in a chain, each mod 2^(n w) (Section 6.1, 6-Add)."""
    x = add(a, b, threads)[0]
    for y in (a, b, a, b, a):
        x = add(x, y, threads)[0]
    return x


def poly(a, b, threads: int = 0):
    """(a a + b) (b b + b) + a b mod 2^(n w) (Section 6.1, Poly)."""
    s1 = add(_mul_low(a, a, threads), b, threads)[0]
    s2 = add(_mul_low(b, b, threads), b, threads)[0]
    return add(_mul_low(s1, s2, threads), _mul_low(a, b, threads), threads)[0]


# ------------------------------------------------------------ conversions
def to_int(limbs) -> int:
    """Python integer of one little-endian limb vector (uint32 or uint64)."""
    x = np.ascontiguousarray(np.asarray(limbs))
    return int.from_bytes(x.tobytes(), "little")


def from_int(v: int, n: int, dtype=np.uint32) -> np.ndarray:
    w = np.dtype(dtype).itemsize
    return np.frombuffer(v.to_bytes(n * w, "little"), dtype=dtype).copy()
