"""Host-side checks of the C ABI (no GPU needed): exported symbols, status
strings and argument validation, which runs before any HIP call."""
from __future__ import annotations

import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def B():
    import paper_2405_14642_amd as B
    return B


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "bigint.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w]+\s*\*?\s*(bi\w+|big\w+)\s*\(", src, flags=re.M)))


def test_header_symbols_exported(B):
    names = _declared_functions()
    assert set(names) >= {"bigadd", "bigmul", "bigadd_v", "bigmul_v", "bi_ctx_create"}
    for n in names:
        assert hasattr(B.lib, n), f"{n} declared in include/bigint.h but not exported"
    assert set(B.EXPORTS) == set(names)


def test_status_strings(B):
    for code in range(-8, 1):
        assert B.lib.bi_status_str(code)
    assert B.lib.bi_status_str(-99) == b"unknown status"


FAKE = 0x10000  # never dereferenced: every call below fails validation first


@pytest.mark.parametrize("args,status", [
    (dict(limb_bits=16), -3),
    (dict(limb_bits=0), -3),
    (dict(n=0), -1),
    (dict(n=(1 << 18) // 32 + 1), -2),
    (dict(n=(1 << 18) // 64 + 1, limb_bits=64), -2),
    (dict(batch=1 << 40), -2),
    (dict(a=None), -1),
    (dict(b=None), -1),
    (dict(out=None), -1),
    (dict(a=FAKE + 2), -3),
    (dict(out=FAKE + 4, limb_bits=64), -3),
    (dict(out=FAKE + 4), -4),                     # out partially overlaps a
    (dict(carry=FAKE + 8), -4),                   # carry bytes inside a
    (dict(), -1),                                 # all valid, but ctx is NULL
    (dict(out=FAKE), -1),                         # in-place is allowed: fails only on ctx
])
def test_bigadd_validation(B, args, status):
    p = dict(a=FAKE, b=FAKE + (1 << 24), out=FAKE + (2 << 24), carry=None, n=4, limb_bits=32, batch=8)
    p.update(args)
    st = B.lib.bigadd(None, p["a"], p["b"], p["out"], p["carry"], p["n"], p["limb_bits"], p["batch"], None)
    assert st == status, B.lib.bi_last_error()
    assert B.lib.bi_last_error()


@pytest.mark.parametrize("args,status", [
    (dict(limb_bits=16), -3),
    (dict(n=0), -1),
    (dict(n=(1 << 40) // 32 + 1), -2),
    (dict(n=(1 << 40) // 64 + 1, limb_bits=64), -2),
    (dict(n=1 << 63), -2),
    (dict(a=None), -1),
    (dict(out=None), -1),
    (dict(b=FAKE + 2), -3),
    (dict(out=FAKE + 4), -4),                     # out partially overlaps a
    (dict(b=FAKE + 8, out=FAKE + 8), -4),         # out == b but partially overlaps a
    (dict(carry=FAKE + (1 << 24) + 3), -4),       # carry byte inside b
    (dict(), -1),                                 # all valid, but ctx is NULL
    (dict(out=FAKE), -1),                         # in-place is allowed: fails only on ctx
    (dict(n=(1 << 40) // 32, b=FAKE + (1 << 38), out=FAKE + (1 << 39)), -1),  # largest size passes
])
def test_bigadd_large_validation(B, args, status):
    p = dict(a=FAKE, b=FAKE + (1 << 24), out=FAKE + (2 << 24), carry=None, n=4, limb_bits=32)
    p.update(args)
    st = B.lib.bigadd_large(None, p["a"], p["b"], p["out"], p["carry"], p["n"], p["limb_bits"], None)
    assert st == status, B.lib.bi_last_error()
    assert B.lib.bi_last_error()


@pytest.mark.parametrize("args,status", [
    (dict(limb_bits=16), -3),
    (dict(n=0), -1),
    (dict(n=(1 << 24) // 32 + 1), -2),
    (dict(n=(1 << 24) // 64 + 1, limb_bits=64), -2),
    (dict(a=None), -1),
    (dict(out=None), -1),
    (dict(a=FAKE + 2), -3),
    (dict(out=FAKE + 8), -4),                     # out overlaps a
    (dict(out=FAKE + (1 << 24) - 16), -4),        # out's 2n limbs reach into b
    (dict(), -1),                                 # all valid, but ctx is NULL
    (dict(n=(1 << 24) // 32), -1),                # the largest size passes the size check
    (dict(algo=9), -1),                           # unknown algorithm
    (dict(algo=-1), -1),
    (dict(algo=4), -1),                           # every algorithm runs 2^18-bit blocks: fails only on ctx
    (dict(block=(1 << 16) + 32), -1),
    (dict(block=1 << 16, algo=3), -1),            # valid block and algorithm: fails only on ctx
])
def test_bigmul_large_validation(B, args, status):
    p = dict(a=FAKE, b=FAKE + (1 << 24), out=FAKE + (2 << 24), n=4, limb_bits=32, algo=0, block=0)
    p.update(args)
    st = B.lib.bigmul_large(None, p["a"], p["b"], p["out"], p["n"], p["limb_bits"], p["algo"], p["block"], None)
    assert st == status, B.lib.bi_last_error()
    assert B.lib.bi_last_error()


@pytest.mark.parametrize("args,valid", [
    (dict(block=1 << 14), True),                  # the NTT path (AUTO, NTT) takes blocks of 2^14..2^18 bits
    (dict(block=1 << 15, algo=3), True),
    (dict(block=1 << 13), False),
    (dict(block=1 << 19), False),
    (dict(block=3 << 14), False),
    (dict(n=(1 << 24) // 32, block=1 << 17), False),  # 128 blocks: the column transform takes at most 64
    (dict(n=(1 << 24) // 32, block=1 << 18), True),
    (dict(n=64 * 512 + 1, block=1 << 14), False),
    (dict(n=64 * 512, block=1 << 14), True),
    (dict(block=1 << 15, algo=2), False),         # block products take 2^16..2^18-bit blocks
    (dict(block=1 << 16, algo=2), True),
])
def test_bigmul_large_block_sizes(B, args, valid):
    """Block sizes each path accepts: an invalid one fails on its own
    (BI_EINVAL naming the blocks), a valid one only on the NULL context."""
    p = dict(a=FAKE, b=FAKE + (1 << 24), out=FAKE + (2 << 24), n=4, limb_bits=32, algo=0, block=0)
    p.update(args)
    st = B.lib.bigmul_large(None, p["a"], p["b"], p["out"], p["n"], p["limb_bits"], p["algo"], p["block"], None)
    assert st == -1
    msg = B.lib.bi_last_error().decode()
    assert (msg == "ctx is NULL") == valid, msg


@pytest.mark.parametrize("args,status", [
    (dict(limb_bits=8), -3),
    (dict(n=0), -1),
    (dict(n=8193), -2),
    (dict(algo=9), -1),
    (dict(algo=-1), -1),
    (dict(out=FAKE), -4),                         # product may not alias a
    (dict(out=FAKE + (1 << 24) - 8), -4),         # overlaps b
    (dict(a=FAKE + 1), -3),
    (dict(), -1),
])
def test_bigmul_validation(B, args, status):
    p = dict(a=FAKE, b=FAKE + (1 << 24), out=FAKE + (2 << 24), n=4, limb_bits=32, batch=8, algo=0)
    p.update(args)
    st = B.lib.bigmul(None, p["a"], p["b"], p["out"], p["n"], p["limb_bits"], p["batch"], p["algo"], None)
    assert st == status, B.lib.bi_last_error()


@pytest.mark.parametrize("args,status", [
    (dict(program=0), -1),
    (dict(program=4), -1),
    (dict(limb_bits=16), -3),
    (dict(n=0), -1),
    (dict(n=8193), -2),
    (dict(n=4097, limb_bits=64), -2),
    (dict(out=FAKE), -4),                         # the result may not alias a
    (dict(out=FAKE + (1 << 24) - 8), -4),         # overlaps b
    (dict(b=FAKE + 2), -3),
    (dict(), -1),                                 # all valid, but ctx is NULL
    (dict(program=2), -1),
    (dict(program=3), -1),
])
def test_fused_validation(B, args, status):
    p = dict(program=1, a=FAKE, b=FAKE + (1 << 24), out=FAKE + (2 << 24), n=4, limb_bits=32, batch=8)
    p.update(args)
    st = B.lib.bi_fused(None, p["program"], p["a"], p["b"], p["out"], p["n"], p["limb_bits"], p["batch"], None)
    assert st == status, B.lib.bi_last_error()


def test_valu_schedule_validation(B):
    import ctypes
    q = (ctypes.c_int * 1)(2)
    w = (ctypes.c_int * 1)(1)
    assert B.lib.bi_tune_set_valu(None, q, w, 1) == -1
    assert B.lib.bi_tune_get_valu(None, q, w, 1) == -1


def test_empty_batch_needs_only_ctx(B):
    assert B.lib.bigadd(None, None, None, None, None, 4, 32, 0, None) == -1
    assert B.lib.bigmul(None, None, None, None, 4, 32, 0, 0, None) == -1


def test_ragged_validation(B):
    assert B.lib.bigadd_v(None, FAKE, FAKE, FAKE, None, FAKE, 1, 48, None) == -3
    assert B.lib.bigadd_v(None, FAKE, FAKE, FAKE, None, None, 1, 32, None) == -1
    assert B.lib.bigadd_v(None, FAKE, FAKE, FAKE, None, FAKE + 4, 1, 32, None) == -1
    assert B.lib.bigmul_v(None, FAKE, FAKE, FAKE, FAKE, 1, 32, 7, None) == -1
    assert B.lib.bigmul_v(None, FAKE, FAKE, FAKE, FAKE, 1, 32, 0, None) == -1


def test_binding_raises(B):
    with pytest.raises(B.BigIntError) as e:
        B.bigadd(None, FAKE, FAKE, FAKE + 4, n_limbs=4, limb_bits=32, batch=8, stream=0)
    assert e.value.status == -4


def test_tuning_validation(B):
    import ctypes
    arr = (ctypes.c_int * 10)()
    assert B.lib.bi_autotune(None, None, arr, 10) == -1
    assert B.lib.bi_tune_get(None, arr, 10) == -1
    assert B.lib.bi_tune_set(None, arr, 10) == -1
    assert B.lib.bi_tune_save(None, b"/tmp/x") == -1
    assert B.lib.bi_tune_load(None, b"/tmp/x") == -1


def test_stream_validation_host(B):
    """Stream-mode argument checks that return before any HIP call."""
    import ctypes
    q = ctypes.c_void_p()
    X = 4096
    assert B.lib.bi_stream_open(None, X, 1, X, 1, X, 2, 32, 8, 0, 1, None, ctypes.byref(q)) == -1   # no ctx
    assert B.lib.bi_stream_open(None, X, 1, X, 1, X, 2, 32, 8, 0, 1, None, None) == -1             # no q
    t = ctypes.c_uint64()
    done = ctypes.c_int()
    assert B.lib.bi_stream_submit(None, X, 1, ctypes.byref(t)) == -1
    assert B.lib.bi_stream_poll(None, 0, ctypes.byref(done)) == -1
    assert B.lib.bi_stream_wait(None, 0) == -1
    assert B.lib.bi_stream_close(None) == 0


def test_binding_checks_tensor_arguments(B):
    """The binding rejects tensors too short for the call, limb-width
    mismatches, non-contiguous views and host tensors with ValueError before
    any library call (so a bad tensor can never reach a kernel)."""
    import torch
    a = torch.zeros((4, 8), dtype=torch.int32)
    short = torch.zeros((4, 7), dtype=torch.int32)
    prod = torch.zeros((4, 16), dtype=torch.int32)
    with pytest.raises(ValueError, match="b holds"):
        B.bigmul(None, a, short, prod)
    with pytest.raises(ValueError, match="out holds"):
        B.bigmul(None, a, a, a)                              # the product needs 2n limbs
    with pytest.raises(ValueError, match="out holds"):
        B.bigadd(None, a, a, short)
    with pytest.raises(ValueError, match="carry holds"):
        B.bigadd(None, a, a, a, torch.zeros(3, dtype=torch.uint8))
    with pytest.raises(ValueError, match="byte elements"):
        B.bigadd(None, a, a.to(torch.int64), a)
    with pytest.raises(ValueError, match="contiguous"):
        B.bigadd(None, a, prod[:, :8], a)
    with pytest.raises(ValueError, match="out holds"):
        B.fused(None, B.PROG_POLY, a, a, short)
    x = torch.zeros(100, dtype=torch.int32)
    with pytest.raises(ValueError, match="out holds"):
        B.bigmul_large(None, x, x, torch.zeros(199, dtype=torch.int32))
    with pytest.raises(ValueError, match="b holds"):
        B.bigadd_large(None, x, x[:99], x)
    with pytest.raises(ValueError, match="desc holds"):
        B.bigmul_v(None, x, x, x, torch.zeros(63, dtype=torch.uint8), 2, 32)
    with pytest.raises(ValueError, match="device tensor"):
        B.bigmul(None, a, a, prod)                           # right sizes, host memory


def test_mul_large_plan(B):
    """The default block of bigmul_large: on the NTT path the smallest of at
    least 2^16 bits with at most 32 blocks (2^18 bits up to 64 blocks at
    2^24 bits); block products 2^16 bits up to 2^20-bit operands, 2^18
    above; argument errors as bigmul_large's."""
    for bits, want in ((1 << 19, 1 << 16), (1 << 20, 1 << 16), (1 << 21, 1 << 16), (1 << 22, 1 << 17),
                       ((1 << 22) + 32, 1 << 18), (1 << 24, 1 << 18)):
        bb, k = B.mul_large_plan(bits // 32, 32, 0)
        assert bb == want and k == -(-bits // bb) and k <= 64, (bits, bb, k)
        if bits % 64 == 0:
            assert B.mul_large_plan(bits // 64, 64, 3) == (bb, k)
    assert B.mul_large_plan(1 << 15, 32, 2) == (1 << 16, 16)
    assert B.mul_large_plan((1 << 15) + 1, 32, 5)[0] == 1 << 18
    assert B.lib.bi_mul_large_plan(0, 32, 0, None, None) == -1
    with pytest.raises(B.BigIntError):
        B.mul_large_plan((1 << 19) + 1, 32, 0)   # beyond 2^24 bits
    with pytest.raises(B.BigIntError):
        B.mul_large_plan(100, 48, 0)
    with pytest.raises(B.BigIntError):
        B.mul_large_plan(100, 32, 9)
