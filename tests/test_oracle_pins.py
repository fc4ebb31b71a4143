"""Pins of the CPU oracle (no GPU)."""
from __future__ import annotations

import json
import os
import tempfile

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests import oracle_pins as pins

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("check", pins.ALL_FAST, ids=lambda f: f.__name__)
def test_pin(orc, check):
    check(orc)


def test_golden_add_examples(orc):
    """Worked carry examples of Section 2 (the all-ones case of Fig. 1)."""
    with open(os.path.join(GOLDEN, "add_examples.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        n, w = c["limbs"], c["limb_bits"]
        dt = np.uint32 if w == 32 else np.uint64
        a = O.from_int(int(c["a"], 16), n, dt)[None]
        b = O.from_int(int(c["b"], 16), n, dt)[None]
        out, carry = orc.add(a, b)
        assert O.to_int(out[0]) == int(c["sum"], 16), c["name"]
        assert int(carry[0]) == c["carry"], c["name"]


# sampled pairs of every workload size against Python's bignum
_SIZES = ([("add", b) for b in W.ADD_SWEEP_BITS] + [("mulq", b) for b in W.MULQ_BITS]
          + [("ntt", b) for b, _ in W.NTT_CASES] + [("small", 4096)])


@pytest.mark.parametrize("kind,bits", _SIZES)
def test_workload_sizes_against_python(orc, kind, bits):
    if kind == "add":
        pairs = [0, 1, 2, 3, 5, 8, 13]
        a, b = W.add_sweep_inputs(bits, pairs=pairs)
        pins.check_against_python(orc, a, b, do_mul=bits <= (1 << 14))
        a32, b32 = W.add_sweep_inputs(bits, pairs=pairs, limb_bits=32)
        pins.check_against_python(orc, a32, b32, do_mul=False)
    elif kind == "mulq":
        a, b = W.mul_quad_inputs(bits, pairs=[0, 7])
        pins.check_against_python(orc, a, b)
    elif kind == "ntt":
        batch = dict(W.NTT_CASES)[bits]
        a, b = W.ntt_inputs(bits, batch, pairs=[0, batch - 1])
        pins.check_against_python(orc, a, b, do_mul=bits <= (1 << 16))
    else:
        a, b = W.small_inputs()
        pins.check_against_python(orc, a[:8], b[:8])


def test_mul_2p18_against_python(orc):
    a, b = W.ntt_inputs(1 << 18, 64, pairs=[3])
    prod = orc.mul(a, b)
    assert O.to_int(prod[0]) == O.to_int(a[0]) * O.to_int(b[0])


# --------------------------------------------------------- planted mistakes
# Each mutation is a plausible slip in the oracle's source; the pins above must
# catch every one of them when run against the mutated copy.
MUTATIONS = {
    "add_dropped_carry": ("carry = s >> 32;", "carry = 0;"),
    "add_wrong_index": ("(uint64_t)b[i] + carry", "(uint64_t)b[n - 1 - i] + carry"),
    "add_carry_shift": ("carry = s >> 32;", "carry = s >> 31;"),
    "mul_wrong_operand": ("(uint64_t)a[i] * (uint64_t)b[j]", "(uint64_t)a[i] * (uint64_t)b[i]"),
    "mul_transposed_index": ("(uint64_t)out[i + j] + carry;\n            out[i + j]", "(uint64_t)out[i + j] + carry;\n            out[j]"),
    "mul_dropped_carry_term": ("(uint64_t)out[i + j] + carry;", "(uint64_t)out[i + j];"),
    "mul_top_limb_offset": ("out[i + n] = (uint32_t)carry;", "out[i + n - 1] += (uint32_t)carry;"),
    "add_ragged_b_offset": ("add_one(a + a_off[p], b + b_off[p]", "add_one(a + a_off[p], b + a_off[p]"),
    "add_ragged_out_offset": ("b + b_off[p], out + out_off[p], n[p]);\n        if", "b + b_off[p], out + a_off[p], n[p]);\n        if"),
    "mul_ragged_b_offset": ("mul_one(a + a_off[p], b + b_off[p]", "mul_one(a + a_off[p], b + a_off[p]"),
    "mul_truncated_row": ("for (size_t j = 0; j < n; ++j) {\n            uint64_t t", "for (size_t j = 0; j + 1 < n; ++j) {\n            uint64_t t"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name):
    old, new = MUTATIONS[name]
    with open(O.SOURCE) as f:
        src = f.read()
    assert src.count(old) >= 1, f"mutation anchor for {name} not found"
    bad = src.replace(old, new, 1)
    with tempfile.TemporaryDirectory() as d:
        cpath = os.path.join(d, "mut.c")
        with open(cpath, "w") as f:
            f.write(bad)
        lib = O.compile_source(cpath, os.path.join(d, "libmut.so"))
        mut = O.Oracle(lib)
        caught = []
        for check in pins.ALL_FAST:
            try:
                check(mut)
            except AssertionError:
                caught.append(check.__name__)
        assert caught, f"planted mistake {name} passed every pin"


@pytest.mark.parametrize("dt", [np.uint32, np.uint64])
@pytest.mark.parametrize("n", [1, 2, 3, 8, 33, 128])
def test_fused_programs_against_python(dt, n):
    """Section 6.1 programs: 6-Add equals the closed form 4a + 3b mod 2^N (a
    different computation from the oracle's chain of additions), Poly equals
    Python's own bignum arithmetic; carry-heavy rows (all ones) included."""
    rng = np.random.default_rng(n)
    info = np.iinfo(dt)
    a = rng.integers(0, info.max, (4, n), dtype=dt, endpoint=True)
    b = rng.integers(0, info.max, (4, n), dtype=dt, endpoint=True)
    a[0] = b[0] = info.max
    a[1] = info.max
    b[1] = 0
    b[1, 0] = 1
    M = 1 << (n * 8 * np.dtype(dt).itemsize)
    got6, gotp, gotm = O.add6(a, b), O.poly(a, b), O.mul_low(a, b)
    for i in range(a.shape[0]):
        A, B = O.to_int(a[i]), O.to_int(b[i])
        assert O.to_int(gotm[i]) == (A * B) % M
        assert O.to_int(got6[i]) == (4 * A + 3 * B) % M
        assert O.to_int(gotp[i]) == ((A * A + B) * (B * B + B) + A * B) % M
