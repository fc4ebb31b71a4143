"""Stream mode (bi_stream_*): bursts of ragged products replayed through a
captured HIP graph (and without one) are bit-exact against the oracle, and
every replay matches the eager bigmul_v result, with unrelated eager work and
synchronisations between the replays."""
from __future__ import annotations

import numpy as np
import pytest

from tests import gpu_util as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import paper_2405_14642_amd as B
    return B


@pytest.fixture(scope="module")
def ctx(B):
    c = B.Context(0)
    yield c
    c.close()


def _problem(seed, count):
    rng = np.random.default_rng(seed)
    u = rng.uniform(0, 13, count)
    ns = np.maximum(1, np.rint(2.0 ** u)).astype(np.int64)  # 1 .. 8192 limbs
    ns[:3] = (1, 8192, 1024)
    tot = int(ns.sum())
    A = rng.integers(0, 2**32, tot, dtype=np.uint32, endpoint=False)
    Bv = rng.integers(0, 2**32, tot, dtype=np.uint32, endpoint=False)
    off = np.concatenate([[0], np.cumsum(ns)[:-1]]).astype(np.uint64)
    A[int(off[3]): int(off[3] + ns[3])] = 0xFFFFFFFF      # one all-ones pair
    Bv[int(off[3]): int(off[3] + ns[3])] = 0xFFFFFFFF
    out_off = np.concatenate([[0], np.cumsum(2 * ns + 1)[:-1]]).astype(np.uint64)
    out_len = int(out_off[-1] + 2 * ns[-1] + 1)
    d = np.zeros(count, dtype=G.DESC_DTYPE)
    d["a_off"], d["b_off"], d["out_off"], d["n_limbs"] = off, off, out_off, ns
    return A, Bv, d, out_len


def _eager_work(B, ctx):
    """Unrelated stream work between graph replays."""
    import torch
    x = torch.full((64, 64), -1, dtype=torch.int32, device="cuda")
    y = torch.empty_like(x)
    B.bigadd(ctx, x, x, y)
    torch.cuda.synchronize()


@pytest.mark.parametrize("use_graph", [True, False])
@pytest.mark.parametrize("algo", [0, 1, 3, 4, 5])
def test_stream_bursts(B, ctx, orc, use_graph, algo):
    count = 120
    A, Bv, d, out_len = _problem(7 + algo, count)
    dA, dB = G.to_dev(A), G.to_dev(Bv)
    ref = G.empty_dev((out_len,), np.uint32)
    ref.zero_()
    B.bigmul_v(ctx, dA, dB, ref, G.desc_dev(d["a_off"], d["b_off"], d["out_off"], d["n_limbs"]), count, 32,
               algo=algo)
    G.sync()
    want_all = G.from_dev(ref, np.uint32)
    for i in range(count):
        n, ao, oo = int(d["n_limbs"][i]), int(d["a_off"][i]), int(d["out_off"][i])
        want = orc.mul(A[ao: ao + n][None], Bv[ao: ao + n][None])[0]
        assert (want_all[oo: oo + 2 * n] == want).all(), ("eager", i, n)

    out = G.empty_dev((out_len,), np.uint32)
    out.zero_()
    bursts = [1, 7, 30, 2, 64, 16]
    assert sum(bursts) == count
    with B.StreamQueue(ctx, dA, dB, out, 32, max_descs=64, algo=algo, use_graph=use_graph) as q:
        start = 0
        tickets = []
        for k, bs in enumerate(bursts):
            t = q.submit(d[start: start + bs])
            tickets.append((t, start, bs))
            if k % 2 == 1:
                q.wait(t)
                assert q.poll(t)
                _eager_work(B, ctx)
            start += bs
        for t, s0, bs in tickets:
            q.wait(t)
            assert q.poll(t)
            got = G.from_dev(out, np.uint32)
            for i in range(s0, s0 + bs):
                n, oo = int(d["n_limbs"][i]), int(d["out_off"][i])
                assert (got[oo: oo + 2 * n] == want_all[oo: oo + 2 * n]).all(), ("burst", t, i, n)
        # the same bursts again into a cleared buffer: every replay matches
        out.zero_()
        G.sync()
        for k, bs in enumerate(bursts[::-1]):
            s0 = count - sum(bursts[::-1][: k + 1])
            t = q.submit(d[s0: s0 + bs])
            q.wait(t)
            got = G.from_dev(out, np.uint32)
            for i in range(s0, s0 + bs):
                n, oo = int(d["n_limbs"][i]), int(d["out_off"][i])
                assert (got[oo: oo + 2 * n] == want_all[oo: oo + 2 * n]).all(), ("replay", k, i, n)
            _eager_work(B, ctx)


def test_stream_validation(B, ctx):
    A, Bv, d, out_len = _problem(3, 8)
    dA, dB = G.to_dev(A), G.to_dev(Bv)
    out = G.empty_dev((out_len,), np.uint32)
    with B.StreamQueue(ctx, dA, dB, out, 32, max_descs=8) as q:
        bad = d.copy()
        bad["out_off"][2] = out_len - 1                 # output range past the buffer
        with pytest.raises(B.BigIntError) as e:
            q.submit(bad)
        assert e.value.status == -1
        bad = d.copy()
        bad["n_limbs"][0] = 8193                        # above 2^18 bits
        with pytest.raises(B.BigIntError) as e:
            q.submit(bad)
        assert e.value.status == -2
        bad = d.copy()
        bad["reserved"][1] = 1
        with pytest.raises(B.BigIntError):
            q.submit(bad)
        with pytest.raises(B.BigIntError) as e:
            q.submit(np.concatenate([d, d]))            # more than max_descs
        assert e.value.status == -2
        with pytest.raises(B.BigIntError):
            q.poll(0)                                   # nothing was issued
        t = q.submit(d)
        q.wait(t)
        assert t == 0 and q.poll(t)


@pytest.mark.parametrize("use_graph", [True, False])
def test_stream_u64_limbs(B, ctx, orc, use_graph):
    """64-bit limbs: classes come from n_limbs * 2 words (device binning with
    a graph, host binning without), products bit-exact against the oracle."""
    rng = np.random.default_rng(64)
    count = 48
    ns = np.maximum(1, np.rint(2.0 ** rng.uniform(0, 12, count))).astype(np.int64)  # 1 .. 4096 u64 limbs
    ns[:4] = (1, 4096, 8, 2048)
    tot = int(ns.sum())
    A = rng.integers(0, 2**64, tot, dtype=np.uint64, endpoint=False)
    Bv = rng.integers(0, 2**64, tot, dtype=np.uint64, endpoint=False)
    off = np.concatenate([[0], np.cumsum(ns)[:-1]]).astype(np.uint64)
    out_off = 2 * off
    d = np.zeros(count, dtype=G.DESC_DTYPE)
    d["a_off"], d["b_off"], d["out_off"], d["n_limbs"] = off, off, out_off, ns
    dA, dB = G.to_dev(A), G.to_dev(Bv)
    out = G.empty_dev((2 * tot,), np.uint64)
    out.zero_()
    with B.StreamQueue(ctx, dA, dB, out, 64, max_descs=32, use_graph=use_graph) as q:
        t0 = q.submit(d[:32])
        t1 = q.submit(d[32:])
        q.wait(t0)
        q.wait(t1)
    got = G.from_dev(out, np.uint64)
    for i in range(count):
        n, ao, oo = int(ns[i]), int(off[i]), int(out_off[i])
        want = orc.mul(A[ao: ao + n][None], Bv[ao: ao + n][None])[0]
        assert (got[oo: oo + 2 * n] == want).all(), (i, n)


@pytest.fixture(scope="module")
def stream_workload(orc):
    """The mixed-size stream at full size (10^5 pairs, 2^10..2^18 bits, 10 %
    all-ones, in its log-uniform bursts) and the oracle's product of every
    pair, laid out as the queue writes them (pair i at 2 off[i])."""
    import workloads as W
    count = 100000
    n, ones = W.stream_sizes(count)
    bursts = W.stream_bursts(count)
    a, b, off = W.stream_inputs(np.arange(count), n, ones)
    nn = n.astype(np.int64)
    prods = orc.mul_ragged([(a[int(o): int(o) + k], b[int(o): int(o) + k]) for o, k in zip(off, nn)])
    want = np.concatenate(prods)
    return a, b, off, nn, bursts, want


@pytest.mark.timeout(900)
@pytest.mark.parametrize("use_graph", [True, False])
def test_stream_full_workload(B, ctx, stream_workload, use_graph):
    """Every one of the 10^5 products of the stream workload, submitted burst
    by burst through the queue (graph replay with device binning, or host
    binning), equals the oracle's."""
    a, b, off, nn, bursts, want = stream_workload
    count = len(nn)
    d = np.zeros(count, dtype=G.DESC_DTYPE)
    d["a_off"], d["b_off"], d["out_off"], d["n_limbs"] = off, off, 2 * off, nn
    dA, dB = G.to_dev(a), G.to_dev(b)
    out = G.empty_dev((2 * int(nn.sum()),), np.uint32)
    out.fill_(-1)
    start = 0
    with B.StreamQueue(ctx, dA, dB, out, 32, max_descs=int(bursts.max()), algo=0, use_graph=use_graph) as q:
        for bs in bursts.tolist():
            q.submit(d[start: start + bs])
            start += bs
        assert start == count
    got = G.from_dev(out, np.uint32)
    bad = np.nonzero(got != want)[0]
    if bad.size:
        pair = np.searchsorted(2 * off.astype(np.int64), bad[:8], side="right") - 1
        raise AssertionError(f"{bad.size} words differ, first in pairs {sorted(set(pair.tolist()))}")
