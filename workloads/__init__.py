"""Seeded synthetic inputs for the batched big-integer workloads.

This module is shared by the CPU oracle tests and by the HIP path (tests,
smoke run, benchmark).  It contains no big-integer arithmetic: it produces
pseudo-random limb arrays and the fixed input patterns (all-ones, carry-heavy)
that the workloads call for.  Every word is a pure function of
(seed, config id, pair index, operand, word index), so any single pair can be
regenerated on its own for sampled checks.

The paper benchmarks on synthetic batches whose total size is fixed
(NumBits * NumInsts = 2^32, Section 6.1); nothing here comes from a dataset.

Workloads (sizes in bits; limbs little-endian, instance-major, contiguous):

* ``small``      256 pairs of 4096-bit integers, u32 limbs, uniform.
* ``add_sweep``  2^10..2^18 bits, u64 limbs, 2^32/N pairs (1 GiB of a+b);
                 75 % uniform, 25 % carry-heavy (a = all-ones, b = 1 or a few
                 uniform low limbs) so carries run the full length.
* ``mul_quad``   2^12..2^15 bits, u32 limbs, 2^25/n pairs (2^26 input limbs).
* ``mul_ntt``    (2^15, 4096), (2^16, 1024), (2^17, 256), (2^18, 64) pairs.
* ``stream``     mixed-size pairs, n = max(1, round(2^u / 32)), u ~ U[10, 18];
                 90 % uniform, 10 % a = b = all-ones.
* ``add_large``  ONE pair of 2^20..2^34-bit integers (the add sweep's 2^32 bits
                 of a+b as a single instance at 2^32), u32 limbs, uniform;
                 pattern variants for tests: ``ripple`` (a = all-ones, b = 1:
                 the carry crosses every limb), ``chains`` (b = ~a except a
                 seeded 1/4096 of the limbs, which are uniform: carry chains
                 of thousands of limbs, many spanning whole tiles).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libwlgen.so")

DEFAULT_SEED = 0x240514642
EXTRA_SEEDS = (0x5EED0001, 0x5EED0002)

CFG_SMALL, CFG_ADD, CFG_MULQ, CFG_NTT, CFG_STREAM, CFG_LARGE = 1, 2, 3, 4, 5, 6

ADD_SWEEP_BITS = (1 << 10, 1 << 12, 1 << 14, 1 << 16, 1 << 18)
MULQ_BITS = (1 << 12, 1 << 13, 1 << 14, 1 << 15)
NTT_CASES = ((1 << 15, 4096), (1 << 16, 1024), (1 << 17, 256), (1 << 18, 64))
MAX_BITS = 1 << 18
LARGE_ADD_BITS = (1 << 20, 1 << 24, 1 << 28, 1 << 32, 1 << 34)

_GAMMA = 0x9E3779B97F4A7C15
_STEP = 0xD1B54A32D192ED03
_M64 = (1 << 64) - 1


def build(force: bool = False) -> str:
    """Compile the generator with gcc (OpenMP) into workloads/libwlgen.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _get():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.wl_fill.argtypes = [ctypes.c_uint64] * 3 + [ctypes.c_void_p] + [ctypes.c_uint64] * 3 + [ctypes.c_void_p]
        lib.wl_fill.restype = None
        lib.wl_key.argtypes = [ctypes.c_uint64] * 4
        lib.wl_key.restype = ctypes.c_uint64
        lib.wl_hash.argtypes = [ctypes.c_uint64]
        lib.wl_hash.restype = ctypes.c_uint64
        lib.wl_fill_ragged.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_uint64,
                                       ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.wl_fill_ragged.restype = None
        _lib = lib
    return _lib


# ---------------------------------------------------------------- reference
def sm64_py(x: int) -> int:
    """SplitMix64 output function on x + gamma (pure Python, for pins)."""
    z = (x + _GAMMA) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def key_py(seed: int, cfg: int, pair: int, operand: int) -> int:
    return sm64_py(sm64_py(seed ^ sm64_py(cfg)) ^ ((2 * pair + operand) & _M64))


def word_py(key: int, j: int) -> int:
    return sm64_py((key + j * _STEP) & _M64)


# ---------------------------------------------------------------- fast path
def words(seed: int, cfg: int, operand: int, nwords: int, pair0: int = 0,
          npairs: int | None = None, pairs=None) -> np.ndarray:
    """(npairs, nwords) uint64 array of generator words for consecutive pairs
    starting at pair0, or for the explicit pair indices in `pairs`."""
    lib = _get()
    if pairs is not None:
        pairs = np.ascontiguousarray(np.asarray(pairs, dtype=np.uint64))
        npairs = pairs.shape[0]
        pptr = pairs.ctypes.data
    else:
        pptr = None
    out = np.empty((npairs, nwords), dtype=np.uint64)
    if npairs and nwords:
        lib.wl_fill(seed & _M64, cfg, pair0, pptr, npairs, operand, nwords, out.ctypes.data)
    return out


def hash64(x: int) -> int:
    return _get().wl_hash(x & _M64)


def pair_hash(seed: int, cfg: int, pair: int) -> int:
    """Per-pair class selector (operand slot 7 is never used for limbs)."""
    return _get().wl_hash(_get().wl_key(seed & _M64, cfg, pair, 7))


def pair_hashes(seed: int, cfg: int, pair_idx: np.ndarray) -> np.ndarray:
    """Vectorised pair_hash over an index array (uint64)."""
    w = words(seed, cfg, 7, 1, pairs=pair_idx)
    return w[:, 0]


def limbs_view(w: np.ndarray, n: int, limb_bits: int) -> np.ndarray:
    """First n limbs of width limb_bits from each row of generator words."""
    if limb_bits == 64:
        return np.ascontiguousarray(w[:, :n])
    if limb_bits == 32:
        return np.ascontiguousarray(w.view(np.uint32)[:, :n])
    raise ValueError("limb_bits must be 32 or 64")


def uniform(seed: int, cfg: int, operand: int, n: int, limb_bits: int,
            pair0: int = 0, npairs: int | None = None, pairs=None) -> np.ndarray:
    nwords = (n * limb_bits + 63) // 64
    return limbs_view(words(seed, cfg, operand, nwords, pair0, npairs, pairs), n, limb_bits)


# ---------------------------------------------------------------- workloads
def small_inputs(seed: int = DEFAULT_SEED):
    """256 pairs of 4096-bit integers in 128 u32 limbs, uniform."""
    a = uniform(seed, CFG_SMALL, 0, 128, 32, 0, 256)
    b = uniform(seed, CFG_SMALL, 1, 128, 32, 0, 256)
    return a, b


def add_sweep_pairs(bits: int) -> int:
    return (1 << 32) // bits


def add_sweep_inputs(bits: int, seed: int = DEFAULT_SEED, pairs=None, limb_bits: int = 64):
    """Addition bandwidth sweep at one size: (a, b) as (npairs, n) arrays.

    pairs=None gives the full batch of 2^32/bits pairs; otherwise the listed
    pair indices (for sampled checks).  A pair is carry-heavy when its class
    hash is 0 mod 4: then a = all-ones and b is either 1 (hash bit 2 set) or
    has ceil(n/8) uniform low limbs and zero above, so the carry out of b's
    lowest nonzero limb runs through every remaining limb of a.
    """
    n = bits // limb_bits
    if pairs is None:
        idx = np.arange(add_sweep_pairs(bits), dtype=np.uint64)
        a = uniform(seed, CFG_ADD, 0, n, limb_bits, 0, idx.shape[0])
        b = uniform(seed, CFG_ADD, 1, n, limb_bits, 0, idx.shape[0])
    else:
        idx = np.asarray(pairs, dtype=np.uint64)
        a = uniform(seed, CFG_ADD, 0, n, limb_bits, pairs=idx)
        b = uniform(seed, CFG_ADD, 1, n, limb_bits, pairs=idx)
    h = pair_hashes(seed, CFG_ADD, idx)
    heavy = (h & np.uint64(3)) == 0
    one = heavy & (((h >> np.uint64(2)) & np.uint64(1)) == 1)
    low = heavy & ~one
    maxv = np.iinfo(a.dtype).max
    a[heavy] = maxv
    b[one] = 0
    b[one, 0] = 1
    k = (n + 7) // 8
    b[np.ix_(low, np.arange(k, n))] = 0
    return a, b


def large_add_inputs(n: int, pattern: str = "uniform", seed: int = DEFAULT_SEED, limb_bits: int = 32):
    """One pair (a, b) of n-limb integers as 1-D arrays (pattern: uniform,
    ripple or chains; see the module docstring)."""
    dt = np.uint32 if limb_bits == 32 else np.uint64
    if pattern == "ripple":
        a = np.full(n, np.iinfo(dt).max, dtype=dt)
        b = np.zeros(n, dtype=dt)
        b[0] = 1
        return a, b
    a = uniform(seed, CFG_LARGE, 0, n, limb_bits, 0, 1)[0]
    if pattern == "uniform":
        return a, uniform(seed, CFG_LARGE, 1, n, limb_bits, 0, 1)[0]
    if pattern == "chains":
        b = ~a
        r = uniform(seed, CFG_LARGE, 1, n, limb_bits, 0, 1)[0]
        sel = (uniform(seed, CFG_LARGE, 2, n, 32, 0, 1)[0] & np.uint32(4095)) == 0
        b[sel] = r[sel]
        return a, b
    raise ValueError(f"unknown pattern {pattern!r}")


def mul_quad_pairs(bits: int) -> int:
    return (1 << 25) // (bits // 32)


def mul_quad_inputs(bits: int, seed: int = DEFAULT_SEED, pairs=None):
    """Quadratic-multiplication sizes: u32 limbs, uniform, 2^25/n pairs."""
    n = bits // 32
    if pairs is None:
        cnt = mul_quad_pairs(bits)
        return (uniform(seed, CFG_MULQ, 0, n, 32, 0, cnt), uniform(seed, CFG_MULQ, 1, n, 32, 0, cnt))
    return (uniform(seed, CFG_MULQ, 0, n, 32, pairs=pairs), uniform(seed, CFG_MULQ, 1, n, 32, pairs=pairs))


def ntt_inputs(bits: int, batch: int, seed: int = DEFAULT_SEED, pairs=None):
    """NTT-multiplication sizes: u32 limbs, uniform."""
    n = bits // 32
    cfg = CFG_NTT * 64 + bits.bit_length()
    if pairs is None:
        return (uniform(seed, cfg, 0, n, 32, 0, batch), uniform(seed, cfg, 1, n, 32, 0, batch))
    return (uniform(seed, cfg, 0, n, 32, pairs=pairs), uniform(seed, cfg, 1, n, 32, pairs=pairs))


def stream_sizes(count: int = 100000, seed: int = DEFAULT_SEED):
    """Per-pair limb counts and all-ones flags of the mixed-size stream.

    u is uniform in [10, 18] (from the top 53 bits of the class hash), the
    size in u32 limbs is max(1, round(2^u / 32)); a pair is all-ones when a
    second hash is 0 mod 10.
    """
    idx = np.arange(count, dtype=np.uint64)
    h = pair_hashes(seed, CFG_STREAM, idx)
    u = 10.0 + 8.0 * ((h >> np.uint64(11)).astype(np.float64) / float(1 << 53))
    n = np.maximum(1, np.rint(np.exp2(u) / 32.0)).astype(np.int64)
    h2 = words(seed, CFG_STREAM, 6, 1, pairs=idx)[:, 0]
    ones = (h2 % np.uint64(10)) == 0
    return n, ones


def stream_bursts(count: int = 100000, seed: int = DEFAULT_SEED):
    """Burst sizes: log-uniform integers in [64, 4096] until `count` pairs."""
    sizes = []
    total, k = 0, 0
    while total < count:
        h = hash64(key_py(seed, CFG_STREAM, k, 5))
        u = (h >> 11) / float(1 << 53)
        b = int(round(64 * (4096 / 64) ** u))
        b = min(b, count - total)
        sizes.append(b)
        total += b
        k += 1
    return np.array(sizes, dtype=np.int64)


def stream_inputs(order: np.ndarray, n: np.ndarray, ones: np.ndarray, seed: int = DEFAULT_SEED):
    """Ragged u32 operand arrays of the stream's pairs in the order given
    (a permutation of pair indices): returns (a, b, offsets), pair order[i]
    at limbs [offsets[i], offsets[i] + n[order[i]])."""
    order = np.ascontiguousarray(order.astype(np.uint64))
    nn = n[order.astype(np.int64)].astype(np.uint64)
    nw = (nn + 1) // 2                        # 64-bit generator words per pair
    woff = np.zeros(len(order), dtype=np.uint64)
    woff[1:] = np.cumsum(nw)[:-1]
    total_w = int(nw.sum())
    lib = _get()
    out = []
    for operand in (0, 1):
        buf = np.empty(total_w, dtype=np.uint64)
        lib.wl_fill_ragged(seed & _M64, CFG_STREAM, order.ctypes.data, len(order), operand, nw.ctypes.data,
                           woff.ctypes.data, buf.ctypes.data)
        out.append(buf.view(np.uint32))
    # pack to exactly n limbs per pair (drop the odd padding limb)
    off = np.zeros(len(order), dtype=np.uint64)
    off[1:] = np.cumsum(nn)[:-1]
    total_l = int(nn.sum())
    idx = np.repeat((2 * woff).astype(np.int64) - off.astype(np.int64), nn.astype(np.int64)) + \
        np.arange(total_l, dtype=np.int64)
    a, b = out[0][idx], out[1][idx]
    mask = np.repeat(ones[order.astype(np.int64)], nn.astype(np.int64))
    a[mask] = 0xFFFFFFFF
    b[mask] = 0xFFFFFFFF
    return a, b, off


def stream_pair(i: int, n: int, ones: bool, seed: int = DEFAULT_SEED):
    if ones:
        a = np.full(n, 0xFFFFFFFF, dtype=np.uint32)
        return a, a.copy()
    a = uniform(seed, CFG_STREAM, 0, n, 32, pairs=[i])[0]
    b = uniform(seed, CFG_STREAM, 1, n, 32, pairs=[i])[0]
    return a, b
