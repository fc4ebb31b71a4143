"""Parity of the HIP multiplication kernels with the CPU oracle (bit-exact)."""
from __future__ import annotations

import numpy as np
import pytest

import workloads as W
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

ALGOS = {"valu": 1, "mfma": 2, "ntt": 3, "ntt64": 4, "kara": 5}


@pytest.fixture(scope="module")
def B():
    import paper_2405_14642_amd as B
    return B


@pytest.fixture(scope="module")
def ctx(B):
    c = B.Context(0)
    yield c
    c.close()


def available(B, ctx, algo, n):
    """Whether `algo` runs n-limb products (BI_EALGO otherwise)."""
    a = G.to_dev(np.ones((1, n), np.uint32))
    out = G.empty_dev((1, 2 * n), np.uint32)
    try:
        B.bigmul(ctx, a, a, out, algo=algo)
    except B.BigIntError as e:
        if e.status == -7:
            return False
        raise
    G.sync()
    return True


def run_mul(B, ctx, a, b, algo):
    A, Bt = G.to_dev(a), G.to_dev(b)
    out = G.empty_dev((a.shape[0], 2 * a.shape[1]), a.dtype)
    B.bigmul(ctx, A, Bt, out, algo=algo)
    G.sync()
    return G.from_dev(out, a.dtype)


def check(orc, a, b, got):
    want = orc.mul(a, b)
    bad = np.nonzero((got != want).any(axis=1))[0]
    assert bad.size == 0, f"{bad.size} of {a.shape[0]} products differ, first {bad[:8]}"


def rand(rng, batch, n, dt=np.uint32):
    return rng.integers(0, np.iinfo(dt).max, size=(batch, n), dtype=dt, endpoint=True)


def patterned(rng, batch, n, dt=np.uint32):
    """Random operands with the edge patterns of the method in some rows."""
    a, b = rand(rng, batch, n, dt), rand(rng, batch, n, dt)
    mx = np.iinfo(dt).max
    a[0], b[0] = mx, mx                          # (2^N - 1)^2: every overflow counter in use
    if batch > 1:
        a[1], b[1] = 0, rand(rng, 1, n, dt)[0]   # zero
    if batch > 2:
        a[2] = 0
        a[2, 0] = 1                              # one
    if batch > 3:
        a[3] = np.iinfo(dt).max // 255 * 0x80     # every byte 0x80: balanced digit -128
        b[3] = np.iinfo(dt).max // 255 * 0x7F     # every byte 0x7F: digit 127 (carries run)
    if batch > 4:
        a[4] = 0
        b[4] = 0
        a[4, -1] = mx                            # top limbs only
        b[4, -1] = mx
    return a, b


SIZES = [1, 2, 3, 4, 5, 7, 8, 15, 16, 17, 31, 32, 33, 63, 64, 65, 100, 127, 128, 129, 255, 256, 257,
         505, 511, 512, 513, 1000, 1017, 1023, 1024, 1025, 2047, 2048, 2049, 4095, 4096, 4097, 8191, 8192]


@pytest.mark.parametrize("algo", list(ALGOS))
@pytest.mark.parametrize("n", SIZES)
def test_sizes(B, ctx, orc, algo, n):
    if not available(B, ctx, ALGOS[algo], n):
        pytest.skip(f"{algo} does not run {n}-limb products")
    rng = np.random.default_rng(1000 + n)
    batch = 7 if n <= 2048 else 3
    a, b = patterned(rng, batch, n)
    check(orc, a, b, run_mul(B, ctx, a, b, ALGOS[algo]))


@pytest.mark.parametrize("algo", list(ALGOS))
def test_small_workload(B, ctx, orc, algo):
    a, b = W.small_inputs()
    if not available(B, ctx, ALGOS[algo], a.shape[1]):
        pytest.skip("unavailable")
    check(orc, a, b, run_mul(B, ctx, a, b, ALGOS[algo]))


@pytest.mark.parametrize("algo", list(ALGOS))
def test_u64_limbs(B, ctx, orc, algo):
    rng = np.random.default_rng(77)
    for n in (1, 3, 64, 100, 512):
        if not available(B, ctx, ALGOS[algo], 2 * n):
            continue
        a, b = patterned(rng, 5, n, np.uint64)
        got = run_mul(B, ctx, a, b, ALGOS[algo])
        assert got.dtype == np.uint64 and got.shape == (5, 2 * n)
        check(orc, a, b, got)


@pytest.mark.parametrize("algo", list(ALGOS))
def test_all_ones_closed_form(B, ctx, algo):
    """(2^N - 1)^2 = 2^(2N) - 2^(N+1) + 1, i.e. limbs [1, 0.., 2^32-2, 2^32-1..]."""
    for n in (64, 1000, 8192):
        if not available(B, ctx, ALGOS[algo], n):
            continue
        a = np.full((2, n), 0xFFFFFFFF, np.uint32)
        got = run_mul(B, ctx, a, a, ALGOS[algo])
        exp = np.concatenate([[1], np.zeros(n - 1), [0xFFFFFFFE], np.full(n - 1, 0xFFFFFFFF)]).astype(np.uint32)
        assert (got == exp).all()


KARA_SIZES = [1000, 1025, 1500, 2048, 2049, 3000, 4096, 4097, 6000, 8191, 8192]


def split_halves(x, h):
    """(low h words, high words zero-padded to h) of each row."""
    lo = x[:, :h].copy()
    hi = np.zeros_like(lo)
    hi[:, : x.shape[1] - h] = x[:, h:]
    return lo, hi


@pytest.mark.parametrize("n", KARA_SIZES)
def test_karatsuba_signs_and_borrows(B, ctx, orc, n):
    """Karatsuba's middle term z0 + z2 - s |a0 - a1| |b0 - b1| for every sign
    case at the top split (a0 < a1, a0 > a1, a0 = a1, for a and b
    independently), halves equal at every level (repeated blocks), and
    |a0 - a1| with a borrow through every word (a0 = 2^(32 (h-1)),
    a1 = 1, and the reverse); sizes with one to three levels and with padded
    halves."""
    rng = np.random.default_rng(5000 + n)
    h = ((n + 1) // 2 + 3) // 4 * 4
    rows = []
    base = rand(rng, 1, n)[0]

    def with_halves(lo, hi):
        x = np.zeros(n, np.uint32)
        x[:h] = lo
        x[h:] = hi[: n - h]
        return x

    lo, hi = split_halves(base[None], h)
    lo, hi = lo[0], hi[0]
    big = hi.copy()
    big[n - h - 1] = 0xFFFFFFFF
    small = big.copy()
    small[n - h - 1] = 0xFFFFFFFE
    cases = {"lt": with_halves(small, big), "gt": with_halves(big, small), "eq": with_halves(hi, hi), "rnd": base}
    for ka in cases:
        for kb in cases:
            rows.append((cases[ka], cases[kb]))
    # borrow through every word of |a0 - a1|
    one = np.zeros(h, np.uint32)
    one[0] = 1
    topbit = np.zeros(h, np.uint32)
    topbit[min(h, n - h) - 1] = 1
    rows.append((with_halves(one, topbit), with_halves(topbit, one)))
    rows.append((with_halves(topbit, one), with_halves(topbit, one)))
    # equal halves at every level: one block repeated
    blk = max(1, n // 8)
    rep = np.resize(rand(rng, 1, blk)[0], n).astype(np.uint32)
    rows.append((rep, rep))
    rows.append((rep, base))
    a = np.stack([r[0] for r in rows])
    b = np.stack([r[1] for r in rows])
    check(orc, a, b, run_mul(B, ctx, a, b, ALGOS["kara"]))


@pytest.mark.parametrize("base", [512, 1024, 2048])
def test_karatsuba_bases(B, orc, base):
    """Every Karatsuba base size (levels down to at most 512, 1024 or 2048
    words), uniform batches at sizes that give one to four levels and ragged
    batches through bigmul_v whose instances keep their own level sizes."""
    c = B.Context(0)
    try:
        B.tune_set_kara(c, [base] * B.NUM_CLASSES)
        rng = np.random.default_rng(base)
        for n in (600, 1025, 2047, 2049, 4096, 5000, 8192):
            a, b = patterned(rng, 4, n)
            plan = B.mul_plan(c, n, 32, ALGOS["kara"])
            assert plan["base_limbs"] <= max(base, 4) or plan["kara_levels"] == 4, plan
            check(orc, a, b, run_mul(B, c, a, b, ALGOS["kara"]))
        ns = np.array([1, 5, 700, 1500, 2100, 3000, 4097, 5000, 6500, 8191, 8192, 4200], dtype=np.int64)
        A = rng.integers(0, 2**32, int(ns.sum()), dtype=np.uint64).astype(np.uint32)
        Bv = rng.integers(0, 2**32, int(ns.sum()), dtype=np.uint64).astype(np.uint32)
        A[: int(ns[:3].sum())] = 0xFFFFFFFF
        off = np.concatenate([[0], np.cumsum(ns)[:-1]]).astype(np.uint64)
        out = G.empty_dev((2 * int(ns.sum()),), np.uint32)
        B.bigmul_v(c, G.to_dev(A), G.to_dev(Bv), out, G.desc_dev(off, off, 2 * off, ns), len(ns), 32,
                   algo=ALGOS["kara"])
        G.sync()
        got = G.from_dev(out, np.uint32)
        for i, n in enumerate(ns.tolist()):
            o = int(off[i])
            want = orc.mul(A[o: o + n][None], Bv[o: o + n][None])[0]
            assert (got[2 * o: 2 * o + 2 * n] == want).all(), (base, i, n)
    finally:
        c.close()


def full_size_check(B, ctx, orc, a, b):
    """Every algorithm that runs this size, in the benchmark's launch
    configuration (one uniform bigmul over the whole batch), against the
    oracle's products of every pair (computed once per size)."""
    n = a.shape[1]
    want = orc.mul(a, b)
    A, Bt = G.to_dev(a), G.to_dev(b)
    out = G.empty_dev((a.shape[0], 2 * n), a.dtype)
    ran = []
    for name, algo in ALGOS.items():
        if not available(B, ctx, algo, n):
            continue
        out.fill_(-1)
        B.bigmul(ctx, A, Bt, out, algo=algo)
        G.sync()
        got = G.from_dev(out, a.dtype)
        bad = np.nonzero((got != want).any(axis=1))[0]
        assert bad.size == 0, f"{name}: {bad.size} of {a.shape[0]} products differ, first {bad[:8]}"
        ran.append(name)
    assert ran


@pytest.mark.parametrize("bits", W.MULQ_BITS)
def test_full_size_quadratic(B, ctx, orc, bits):
    """The quadratic-multiplication workload at full size (2^25 / n pairs):
    every product of every algorithm compared with the oracle."""
    a, b = W.mul_quad_inputs(bits)
    full_size_check(B, ctx, orc, a, b)


@pytest.mark.parametrize("bits,batch", W.NTT_CASES)
def test_full_size_ntt_workload(B, ctx, orc, bits, batch):
    """The NTT-multiplication workload at full size: every product of every
    algorithm compared with the oracle."""
    a, b = W.ntt_inputs(bits, batch)
    full_size_check(B, ctx, orc, a, b)


@pytest.mark.parametrize("algo", ["auto"] + list(ALGOS))
@pytest.mark.parametrize("lb", [32, 64])
def test_ragged_bigmul_v(B, ctx, orc, algo, lb):
    """bigmul_v over a ragged batch spanning every size class; b stored in
    reverse instance order, outputs with gaps between them.  A forced
    algorithm applies to the classes it supports, the others use the tuned
    choice."""
    dt = np.uint32 if lb == 32 else np.uint64
    rng = np.random.default_rng(4242 + lb)
    ns = [1, 2, 16, 17, 33, 64, 65, 100, 128, 129, 255, 300, 511, 513, 1000, 1025, 2047, 2049, 4000, 4097, 8192]
    if lb == 64:
        ns = [max(1, n // 2) for n in ns]
    ns = np.array(ns, dtype=np.int64)
    tot = int(ns.sum())
    A = rng.integers(0, np.iinfo(dt).max, tot, dtype=dt, endpoint=True)
    Bv = rng.integers(0, np.iinfo(dt).max, tot, dtype=dt, endpoint=True)
    a_off = np.concatenate([[0], np.cumsum(ns)[:-1]]).astype(np.uint64)
    b_off = np.concatenate([[0], np.cumsum(ns[::-1])[:-1]])[::-1].astype(np.uint64)
    A[: int(ns[0] + ns[1] + ns[2])] = np.iinfo(dt).max          # all-ones operands in the small classes
    Bv[int(b_off[2]): int(b_off[2] + ns[2])] = np.iinfo(dt).max
    out_off = np.concatenate([[0], np.cumsum(2 * ns + 3)[:-1]]).astype(np.uint64)
    out_len = int(out_off[-1] + 2 * ns[-1] + 3)
    dev_out = G.empty_dev((out_len,), dt)
    desc = G.desc_dev(a_off, b_off, out_off, ns)
    code = 0 if algo == "auto" else ALGOS[algo]
    B.bigmul_v(ctx, G.to_dev(A), G.to_dev(Bv), dev_out, desc, len(ns), lb, algo=code)
    G.sync()
    got = G.from_dev(dev_out, dt)
    for i, n in enumerate(ns.tolist()):
        ao, bo, oo = int(a_off[i]), int(b_off[i]), int(out_off[i])
        want = orc.mul(A[ao: ao + n][None], Bv[bo: bo + n][None])[0]
        assert (got[oo: oo + 2 * n] == want).all(), (i, n)


def test_autotune_and_auto_dispatch(B, orc):
    """bi_autotune picks a supported algorithm for every size class, and
    BI_MUL_AUTO with the tuned table stays bit-exact; bi_tune_set rejects an
    entry that names no algorithm (AUTO or an unknown value) and accepts a
    valid table."""
    c = B.Context(0)
    try:
        algos = B.autotune(c)
        assert len(algos) == B.NUM_CLASSES and all(a in (1, 2, 3, 4, 5) for a in algos)
        assert B.tune_get(c) == algos
        ragged = B.tune_get_list(c)
        assert len(ragged) == B.NUM_CLASSES and all(a in (1, 2, 3, 4, 5) for a in ragged)
        with pytest.raises(B.BigIntError):
            B.tune_set_list(c, [9] + [1] * (B.NUM_CLASSES - 1))   # no such algorithm
        assert B.tune_get_list(c) == ragged
        for q, w in B.tune_get_valu(c):
            assert q in (2, 4) and w in (1, 2, 4, 8, 16), (q, w)
        rng = np.random.default_rng(99)
        for n in (16, 100, 700, 3000, 8192):
            a, b = patterned(rng, 3, n)
            check(orc, a, b, run_mul(B, c, a, b, 0))
        for bad in (0, 9):
            with pytest.raises(B.BigIntError):
                B.tune_set(c, [bad] + [1] * (B.NUM_CLASSES - 1))
        assert B.tune_get(c) == algos
        B.tune_set(c, [2] * B.NUM_CLASSES)
        assert B.tune_get(c) == [2] * B.NUM_CLASSES
        B.tune_set(c, [4] * B.NUM_CLASSES)
        assert B.tune_get(c) == [4] * B.NUM_CLASSES
        B.tune_set(c, [1] * B.NUM_CLASSES)
        assert B.tune_get(c) == [1] * B.NUM_CLASSES
    finally:
        c.close()


def test_tune_save_load(B, orc, tmp_path):
    """Autotuned tables persist: saved, loaded into a fresh context (the same
    tables, products bit-exact), and a file for another architecture or a
    malformed one is refused with the context unchanged."""
    c = B.Context(0)
    try:
        algos = B.autotune(c)
        valu = B.tune_get_valu(c)
        kara = B.tune_get_kara(c)
        ragged = B.tune_get_list(c)
        assert all(k in (512, 1024, 2048) for k in kara)
        path = str(tmp_path / "tune.txt")
        B.tune_save(c, path)
    finally:
        c.close()
    d = B.Context(0)
    try:
        B.tune_set(d, [1] * B.NUM_CLASSES)
        B.tune_set_kara(d, [512] * B.NUM_CLASSES)
        B.tune_set_list(d, [1] * B.NUM_CLASSES)
        B.tune_load(d, path)
        assert B.tune_get(d) == algos and B.tune_get_valu(d) == valu and B.tune_get_kara(d) == kara
        assert B.tune_get_list(d) == ragged
        rng = np.random.default_rng(7)
        for n in (40, 700, 5000):
            a, b = patterned(rng, 3, n)
            check(orc, a, b, run_mul(B, d, a, b, 0))
        text = open(path).read()
        other = str(tmp_path / "other.txt")
        arch = [l for l in text.splitlines() if l.startswith("arch ")][0]
        open(other, "w").write(text.replace(arch, "arch gfx942"))
        B.tune_set(d, [2] * B.NUM_CLASSES)
        with pytest.raises(B.BigIntError):
            B.tune_load(d, other)
        open(other, "w").write(text.replace("mul_algo", "mul_alg"))
        with pytest.raises(B.BigIntError):
            B.tune_load(d, other)
        with pytest.raises(B.BigIntError):
            B.tune_load(d, str(tmp_path / "missing.txt"))
        assert B.tune_get(d) == [2] * B.NUM_CLASSES
        # a version-1 file (no Karatsuba bases) loads with the default base
        v1 = "\n".join(l for l in text.splitlines() if not l.startswith(("kara_base", "list_algo"))).replace(
            "bigint-tune 2", "bigint-tune 1")
        open(other, "w").write(v1 + "\n")
        B.tune_load(d, other)
        assert B.tune_get(d) == algos and B.tune_get_kara(d) == [1024] * B.NUM_CLASSES
        assert B.tune_get_list(d) == algos  # a version-1 file's table serves ragged batches too
        open(other, "w").write(text.replace("kara_base 512", "kara_base 500").replace("kara_base 1024", "kara_base 1000")
                               .replace("kara_base 2048", "kara_base 2000"))
        with pytest.raises(B.BigIntError):
            B.tune_load(d, other)
        with pytest.raises(B.BigIntError):
            B.tune_set_kara(d, [1000] + [1024] * (B.NUM_CLASSES - 1))
        assert B.tune_get_kara(d) == [1024] * B.NUM_CLASSES
    finally:
        d.close()


def test_valu_schedules(B, orc):
    """Every VALU schoolbook schedule (Q = 2 or 4 output words per lane, 1..16
    waves) that fits a class's sizes is bit-exact, for the class's largest
    size and a smaller one, uniform and ragged; invalid ones are rejected."""
    c = B.Context(0)
    try:
        rng = np.random.default_rng(123)
        for k in range(B.NUM_CLASSES):
            nmax = 16 << k
            sizes = [nmax, nmax // 2 + 1] if k else [16, 5]
            for q in (2, 4):
                for w in (1, 2, 4, 8, 16):
                    sched = [(0, 0)] * B.NUM_CLASSES
                    sched[k] = (q, w)
                    try:
                        B.tune_set_valu(c, sched)
                    except B.BigIntError as e:
                        assert e.status == -1
                        continue
                    assert B.tune_get_valu(c)[k] == (q, w)
                    for n in sizes:
                        a, b = patterned(rng, 3, n)
                        check(orc, a, b, run_mul(B, c, a, b, 1))
                    # ragged: one class, two sizes, through bigmul_v
                    ns = np.array(sizes, dtype=np.int64)
                    A = rng.integers(0, 2**32, int(ns.sum()), dtype=np.uint32)
                    Bv = rng.integers(0, 2**32, int(ns.sum()), dtype=np.uint32)
                    off = np.concatenate([[0], np.cumsum(ns)[:-1]]).astype(np.uint64)
                    oo = 2 * off
                    out = G.empty_dev((2 * int(ns.sum()),), np.uint32)
                    B.bigmul_v(c, G.to_dev(A), G.to_dev(Bv), out, G.desc_dev(off, off, oo, ns), len(ns), 32, algo=1)
                    G.sync()
                    got = G.from_dev(out, np.uint32)
                    for i, n in enumerate(ns.tolist()):
                        o = int(off[i])
                        want = orc.mul(A[o: o + n][None], Bv[o: o + n][None])[0]
                        assert (got[2 * o: 2 * o + 2 * n] == want).all(), (k, q, w, n)
        with pytest.raises(B.BigIntError):
            B.tune_set_valu(c, [(3, 1)] + [(0, 0)] * (B.NUM_CLASSES - 1))
        with pytest.raises(B.BigIntError):
            B.tune_set_valu(c, [(2, 3)] + [(0, 0)] * (B.NUM_CLASSES - 1))
    finally:
        c.close()
