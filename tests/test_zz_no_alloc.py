"""bigmul_noalloc, the entry point for callers that cannot allocate device
memory (every scratch buffer in the library's fixed per-GPU array), called
through the C ABI and compared bit-exactly with bigmul's products: per
algorithm, two calls in a row, the second with a smaller input (the array
keeps the first call's contents), batches large enough to run in rounds of
the array, and a few products against the oracle."""
from __future__ import annotations

import numpy as np
import pytest

from tests import gpu_util as G

pytestmark = pytest.mark.gpu

# (algorithm, (n, batch) of the first call, (n, batch) of the second)
CASES = [
    (3, (8192, 300), (2048, 17)),   # NTT: 300 x 512 KiB of transforms run in rounds of the array
    (4, (8192, 200), (1000, 9)),    # PrimeField64 NTT
    (2, (8192, 40), (3000, 5)),     # MFMA large-product slots
    (5, (8192, 100), (1500, 7)),    # Karatsuba levels (and their base) in rounds
    (1, (700, 33), (65, 3)),        # VALU schoolbook (no scratch)
    (0, (8192, 64), (4096, 8)),     # the tuned choice
]


@pytest.fixture(scope="module")
def B():
    import paper_2405_14642_amd as B
    return B


@pytest.fixture(scope="module")
def ctx(B):
    c = B.Context(0)
    yield c
    c.close()


def noalloc(B, ctx, A, Bt, out, n, batch, algo):
    import torch
    st = B.lib.bigmul_noalloc(ctx.handle, A.data_ptr(), Bt.data_ptr(), out.data_ptr(), n, 32, batch, algo,
                              torch.cuda.current_stream().cuda_stream)
    assert st == 0, B.lib.bi_last_error().decode()


@pytest.mark.parametrize("algo,first,second", CASES)
def test_noalloc_matches_bigmul(B, ctx, orc, algo, first, second):
    for k, (n, batch) in enumerate((first, second)):
        rng = np.random.default_rng(31 * algo + k)
        a = rng.integers(0, 2**32, (batch, n), dtype=np.uint64).astype(np.uint32)
        b = rng.integers(0, 2**32, (batch, n), dtype=np.uint64).astype(np.uint32)
        a[0] = 0xFFFFFFFF
        b[0] = 0xFFFFFFFF
        A, Bt = G.to_dev(a), G.to_dev(b)
        ref = G.empty_dev((batch, 2 * n), np.uint32)
        B.bigmul(ctx, A, Bt, ref, algo=algo)
        out = G.empty_dev((batch, 2 * n), np.uint32)
        out.fill_(-1)
        noalloc(B, ctx, A, Bt, out, n, batch, algo)
        G.sync()
        got, want = G.from_dev(out, np.uint32), G.from_dev(ref, np.uint32)
        bad = np.nonzero((got != want).any(axis=1))[0]
        assert bad.size == 0, f"call {k}: {bad.size} of {batch} products differ from bigmul, first {bad[:8]}"
        idx = [0, batch // 2, batch - 1]
        assert (got[idx] == orc.mul(a[idx], b[idx])).all(), f"call {k}: products differ from the oracle"
