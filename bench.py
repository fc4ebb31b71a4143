"""Benchmark of the batched big-integer hot path on one MI355X.

Default workload (all): one JSON line carrying
  * the addition bandwidth sweep (the headline value).  One step adds, at
    each of 2^10, 2^12, 2^14, 2^16 and 2^18 bits (u64 limbs), a batch of
    2^32/N pairs (1 GiB of operands, 0.5 GiB of sums per size), i.e. five
    bigadd launches; inputs are seeded (75 % uniform, 25 % carry-heavy);
  * mul_quadratic: 2^12..2^15 bits, 2^25/n pairs, every algorithm, best per
    size, each with its integer-op roofline;
  * mul_ntt: (2^15, 4096), (2^16, 1024), (2^17, 256), (2^18, 64) pairs, the
    same;
  * stream: 10^5 products of mixed sizes in bursts (the stream queue against
    per-class padded launches, saturated throughput and burst latency at 0.8x
    load);
  each with the CPU oracle timed beside it (all cores and one core).
Inputs are generated on the host, copied to HBM once and stay resident; the
timed regions contain only the kernels.  Every launch is timed with HIP
events on the stream it runs on.

Other workloads (--workload) print their own line: add, mulq, ntt, stream
(the parts above alone), copy (a plain 1 GiB device copy, the known-size
kernel that scales the HBM byte counters), fused (the paper's fused programs
6-Add and Poly, Section 6.1, over the addition sweep's batches, with 1-Add
beside them), add_large / mul_large (one integer beyond a workgroup), peaks
(register-resident issue rates of the instructions the rooflines count).

Top-level fields (rank 0, one GPU):
  value   whole-job additions per second over the step (all five sizes);
  roofline   for the dominant addition kernel: algorithmic bytes per launch
             (3 N/8 per pair = 1.5 GiB) over its average launch time,
             against 8 TB/s;
  cpu_baseline   the CPU oracle on this host's cores over the same sweep.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


class G:
    """numpy limb arrays <-> device tensors (torch tensors as raw limb buffers)."""

    @staticmethod
    def to_dev(x):
        import torch
        x = np.ascontiguousarray(x)
        return torch.from_numpy(x.view({4: np.int32, 8: np.int64}[x.dtype.itemsize])).to("cuda")

    @staticmethod
    def empty_dev(shape, dtype):
        import torch
        return torch.empty(shape, dtype=torch.int32 if np.dtype(dtype).itemsize == 4 else torch.int64, device="cuda")


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="all",
                   choices=["all", "add", "add_large", "mul_large", "mulq", "ntt", "stream", "copy", "fused", "peaks"])
    p.add_argument("--stream-pairs", type=int, default=100000, help="pairs in the mixed-size stream")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    p.add_argument("--cpu-seconds", type=float, default=12.0, help="CPU baseline budget")
    p.add_argument("--sizes", default="", help="comma-separated subset of sizes in bits (profiling runs)")
    p.add_argument("--algos", default="valu,mfma,ntt,ntt64,kara", help="multiplication algorithms to time")
    p.add_argument("--graph-replays", action="store_true",
                   help="NTT sizes: also time the best call per size as HIP-graph replays (off by default: a "
                        "capture in the process measured the stream workload's host-binned queue slower)")
    return p.parse_args()


def cpu_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed PMC summary
    (FETCH_SIZE + WRITE_SIZE, scaled by a copy of known size), or None when
    the summary is for another kernel or the add kernels' source changed since
    the counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "bigadd_sweep_traffic.md")
    try:
        text = open(path).read()
        rec = json.loads(re.search(r"```json\s*(\{.*?\})\s*```", text, re.S).group(1))
        src = b"".join(open(os.path.join(ROOT, "paper_2405_14642_amd", "csrc", f), "rb").read()
                       for f in ("bigadd.hip", "bi_common.hpp"))
    except (OSError, AttributeError, ValueError):
        return None
    if rec.get("source_sha256_16") != hashlib.sha256(src).hexdigest()[:16]:
        return None
    for r in rec.get("launches", []):
        if r.get("kernel") == kernel:
            return {"bytes_per_launch": r["traffic_bytes"], "read": r["fetch_bytes"], "written": r["write_bytes"],
                    "source": "profiles/bigadd_sweep_traffic.md"}
    return None


def measured_large_traffic(case):
    """HBM bytes of one bigadd_large call (all four kernels) from the committed
    PMC summary, or None when the case is missing or the kernels' source
    changed since the counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "bigadd_large_traffic.md")
    try:
        text = open(path).read()
        rec = json.loads(re.search(r"```json\s*(\{.*?\})\s*```", text, re.S).group(1))
        src = b"".join(open(os.path.join(ROOT, "paper_2405_14642_amd", "csrc", f), "rb").read()
                       for f in ("bigadd_large.hip", "bi_common.hpp"))
    except (OSError, AttributeError, ValueError):
        return None
    if rec.get("source_sha256_16") != hashlib.sha256(src).hexdigest()[:16]:
        return None
    for r in rec.get("calls", []):
        if r.get("case") == case:
            return r["traffic_bytes"]
    return None


def add_kernel_name(n_limbs, limb_bits):
    """Name of the addition kernel the library launches for this shape (16-byte
    chunks; mirrors the size classes of the launcher in csrc/bigadd.hip)."""
    m = n_limbs * limb_bits // 128
    if m <= 64:
        return "bi::bigadd_packed_kernel<4, 4, true>"
    rows = (m + 63) // 64
    if rows <= 2:
        return "bi::bigadd_multi_kernel<4, 2, 2, true>"
    if rows <= 4:
        return "bi::bigadd_multi_kernel<4, 1, 4, true>"
    u, nw = (1, 2) if rows <= 2 else (1, 4) if rows <= 4 else (2, 4) if rows <= 8 else (2, 8) if rows <= 16 else (4, 8)
    return f"bi::bigadd_coop_kernel<4, {u}, {nw}, true>"


def bench_add(args):
    import torch

    import paper_2405_14642_amd as B
    import workloads as W

    ctx = B.Context(0)
    stream = torch.cuda.current_stream()
    sizes = W.ADD_SWEEP_BITS
    if args.sizes:
        sizes = tuple(int(x) for x in args.sizes.split(","))
    bufs = {}
    for bits in sizes:
        a, b = W.add_sweep_inputs(bits)
        A, Bt = G.to_dev(a), G.to_dev(b)
        out = torch.empty_like(A)
        carry = torch.empty(a.shape[0], dtype=torch.uint8, device="cuda")
        bufs[bits] = (A, Bt, out, carry, a.shape[1], a.shape[0])
        del a, b
    torch.cuda.synchronize()

    def launch(bits):
        A, Bt, out, carry, n, batch = bufs[bits]
        B.bigadd(ctx, A, Bt, out, carry, n_limbs=n, limb_bits=64, batch=batch, stream=stream.cuda_stream)

    for _ in range(args.warmup):
        for bits in sizes:
            launch(bits)
    torch.cuda.synchronize()

    ev = {bits: [] for bits in sizes}
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(args.steps):
        for bits in sizes:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            launch(bits)
            e1.record(stream)
            ev[bits].append((e0, e1))
    t1.record(stream)
    torch.cuda.synchronize()
    total_ms = t0.elapsed_time(t1)
    ms_per_step = total_ms / args.steps

    per_size = {}
    pairs_per_step = 0
    bytes_per_launch = 3 * (1 << 32) // 8  # 3 N/8 bytes per pair x 2^32/N pairs
    for bits in sizes:
        us = 1e3 * float(np.mean([a.elapsed_time(b) for a, b in ev[bits]]))
        pairs = W.add_sweep_pairs(bits)
        pairs_per_step += pairs
        gbs = bytes_per_launch / (us * 1e-6) / 1e9
        per_size[str(bits)] = {"pairs": pairs, "us_per_launch": round(us, 2), "adds_per_s": pairs / (us * 1e-6),
                               "GB_per_s": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
    # Dominant kernel: the one behind the slowest launch of the step (every
    # launch moves the same 1.5 GiB).
    dom_bits = max(sizes, key=lambda b: per_size[str(b)]["us_per_launch"])
    dom_us = per_size[str(dom_bits)]["us_per_launch"]
    achieved = bytes_per_launch / (dom_us * 1e-6) / 1e9
    dom_kernel = add_kernel_name(dom_bits // 64, 64) + f" at 2^{dom_bits.bit_length() - 1} bits"
    tr = measured_traffic(dom_kernel)
    roofline = {"bound": "hbm", "kernel": dom_kernel,
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": tr["bytes_per_launch"] if tr else None,
                "traffic_detail": tr,
                "avg_launch_us": round(dom_us, 2), "algorithmic_bytes_per_launch": bytes_per_launch}
    value = pairs_per_step / (ms_per_step * 1e-3)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline_add(args, W)
    del bufs
    ctx.close()
    return {
        "metric": "bigadd additions/s over the 2^10..2^18-bit sweep (u64 limbs, 1 GiB of operands per size)",
        "value": value, "unit": "adds/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic (seeded splitmix64; 75% uniform, 25% carry-heavy)",
        "config": {"workload": "add_sweep", "sizes_bits": list(sizes), "limb_bits": 64,
                   "pairs": [W.add_sweep_pairs(b) for b in sizes], "operand_bytes_per_size": 1 << 30,
                   "parallelism": "single-gpu"},
        "roofline": roofline, "per_size": per_size, "cpu_baseline": cpu,
    }


# Peak rates used for the multiplication rooflines: 1024 SIMDs x 2.4 GHz x
# the lanes per clock and SIMD of each instruction class, as the register-
# resident issue-rate probe (--workload peaks) measures them on the device:
# v_mad_u64_u32, v_mul_lo_u32, v_mul_hi_u32 and v_addc_co_u32 (VOP3 with
# carry) 16 lanes/clk/SIMD (measured 15.0-15.4), plain 32-bit adds,
# subtracts and min 32 (measured 25.7).
# VALU schoolbook: one v_mad_u64_u32 + one v_addc_co_u32 per 32x32-bit
# product term -> 8 terms/clk/SIMD (the probe's fused term: 7.65).
VALU_MAC_PEAK = 1024 * 8 * 2.4e9                  # 1.97e13 u32 MAC/s
# NTT: a radix-2 butterfly with a Shoup twiddle is 3 multiply-class
# instructions (v_mul_hi_u32, 2 x v_mul_lo_u32) and 9 add-class ones (the
# add, subtract and min of add_mod, sub_mod and the Shoup correction).
NTT_BFLY_PEAK = 1024 * 2.4e9 / (3 / 16 + 9 / 32)  # 5.24e12 butterflies/s
MFMA_I8_PEAK_OPS = 5.0e15                        # dense int8, ops (2 per MAC)
# PrimeField64 NTT: a butterfly with a 64-bit Montgomery twiddle product is
# 7 multiply-class instructions (4 for the 64x64 -> 128-bit product, 3 for the
# reduction by p = 29 2^57 + 1) and 16 add-class ones (64-bit add, subtract,
# compare-select and shifts).
NTT64_BFLY_PEAK = 1024 * 2.4e9 / (7 / 16 + 16 / 32)  # 2.62e12 butterflies/s

ALGO_IDS = {"valu": 1, "mfma": 2, "ntt": 3, "ntt64": 4, "kara": 5}


def mul_ideal_seconds(ctx, n, algo=0):
    """Time of one n-word product at the roofline of the algorithm the
    context runs for it (AUTO: the tuned choice; Karatsuba: its base
    products)."""
    import paper_2405_14642_amd as B
    plan = B.mul_plan(ctx, n, 32, algo)
    name = {v: k for k, v in ALGO_IDS.items()}[plan["base_algo"]]
    return 3 ** plan["kara_levels"] * _unit_seconds(name, plan["base_limbs"])


def _unit_seconds(name, n):
    """Seconds of one n-word product by `name` at its peak (the MFMA one
    against the int8 rate alone)."""
    if name == "valu":
        return float(n) * n / VALU_MAC_PEAK
    if name in ("ntt", "ntt64"):
        m = 11
        while (1 << m) < (4 if name == "ntt" else 2) * n:
            m += 1
        return 2.0 * 3 * (1 << m) / 2 * m / (NTT_BFLY_PEAK if name == "ntt" else NTT64_BFLY_PEAK)
    return 2.0 * (4 * n) ** 2 / MFMA_I8_PEAK_OPS


def mul_roofline(name, n, batch, us):
    """Roofline of `batch` products of n-word operands by algorithm `name`
    that took `us` microseconds."""
    macs = float(batch) * n * n
    if name == "valu":
        return {"bound": "alu", "achieved": round(macs / (us * 1e-6) / 1e12, 3),
                "peak": round(VALU_MAC_PEAK / 1e12, 3), "unit": "T u32-MAC/s",
                "frac": round(macs / (us * 1e-6) / VALU_MAC_PEAK, 4)}
    if name in ("ntt", "ntt64"):
        m = 11
        while (1 << m) < (4 if name == "ntt" else 2) * n:
            m += 1
        bfly = 2.0 * 3 * batch * (1 << m) / 2 * m
        peak = NTT_BFLY_PEAK if name == "ntt" else NTT64_BFLY_PEAK
        return {"bound": "alu", "achieved": round(bfly / (us * 1e-6) / 1e12, 3),
                "peak": round(peak / 1e12, 3),
                "unit": "T butterflies/s" + ("" if name == "ntt" else " (PF64)"),
                "frac": round(bfly / (us * 1e-6) / peak, 4), "butterflies": bfly}
    # mfma: min(int8 peak, arithmetic intensity x HBM); the operands and the
    # product (16 n bytes per pair) bound the small sizes
    ops = 2.0 * batch * (4 * n) ** 2
    hbm_roof = ops / (16.0 * n * batch) * HBM_PEAK_GBS * 1e9
    peak = min(MFMA_I8_PEAK_OPS, hbm_roof)
    return {"bound": "mfma" if peak == MFMA_I8_PEAK_OPS else "hbm",
            "achieved": round(ops / (us * 1e-6) / 1e12, 1), "peak": round(peak / 1e12, 1),
            "unit": "TOP/s (int8)", "frac": round(ops / (us * 1e-6) / peak, 4)}


def bench_mul(args, kind):
    import torch

    import paper_2405_14642_amd as B
    import workloads as W

    ctx = B.Context(0)
    stream = torch.cuda.current_stream()
    if kind == "mulq":
        cases = [(bits, W.mul_quad_pairs(bits)) for bits in W.MULQ_BITS]
        gen = lambda bits, batch: W.mul_quad_inputs(bits)
    else:
        cases = list(W.NTT_CASES)
        gen = lambda bits, batch: W.ntt_inputs(bits, batch)
    if args.sizes:
        keep = {int(x) for x in args.sizes.split(",")}
        cases = [c for c in cases if c[0] in keep]
    algos = [a for a in args.algos.split(",") if a]
    results = {}
    step_ms = 0.0
    step_pairs = 0
    for bits, batch in cases:
        a, b = gen(bits, batch)
        n = a.shape[1]
        A, Bt = G.to_dev(a), G.to_dev(b)
        out = G.empty_dev((batch, 2 * n), np.uint32)
        del a, b
        best = None
        for name in algos:
            algo = ALGO_IDS[name]
            try:
                B.bigmul(ctx, A, Bt, out, algo=algo, stream=stream.cuda_stream)
            except B.BigIntError as e:
                if e.status == -7:
                    continue
                raise
            torch.cuda.synchronize()
            for _ in range(args.warmup):
                B.bigmul(ctx, A, Bt, out, algo=algo, stream=stream.cuda_stream)
            torch.cuda.synchronize()
            # the calls back to back, timed as one region: the average call
            # of a stream of them (throughput), host enqueue overlapped
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(args.steps):
                B.bigmul(ctx, A, Bt, out, algo=algo, stream=stream.cuda_stream)
            e1.record(stream)
            torch.cuda.synchronize()
            us = 1e3 * e0.elapsed_time(e1) / args.steps
            macs = float(batch) * n * n
            r = {"us_per_launch": round(us, 2), "mults_per_s": batch / (us * 1e-6),
                 "u32_macs_per_s": macs / (us * 1e-6)}
            if name == "kara":
                # the work actually done: 3^levels base products per pair with
                # the base algorithm, against that algorithm's roofline
                plan = B.mul_plan(ctx, n, 32, algo)
                nb = batch * 3 ** plan["kara_levels"]
                base_name = {v: k for k, v in ALGO_IDS.items()}[plan["base_algo"]]
                r["plan"] = dict(plan, base_products_per_launch=nb)
                r["roofline"] = mul_roofline(base_name, plan["base_limbs"], nb, us)
                # context: the same products as one full-size int8-MFMA schoolbook
                sb_ops = 2.0 * batch * (4 * n) ** 2
                r["schoolbook_mfma_equiv_frac"] = round(sb_ops / (us * 1e-6) / MFMA_I8_PEAK_OPS, 4)
            else:
                r["roofline"] = mul_roofline(name, n, batch, us)
                if "butterflies" in r["roofline"]:
                    r["butterflies_per_launch"] = r["roofline"].pop("butterflies")
            results.setdefault(str(bits), {})[name] = r
            if best is None or us < best[1]:
                best = (name, us)
        if best:
            results[str(bits)]["best"] = best[0]
            step_ms += best[1] / 1e3
            step_pairs += batch
            if kind == "ntt" and args.graph_replays:
                results[str(bits)]["graph"] = graph_replay_timing(ctx, B, A, Bt, out, ALGO_IDS[best[0]], args.steps)
        del A, Bt, out
    ctx.close()
    last = str(cases[-1][0])
    dom = results[last][results[last]["best"]]
    return {
        "metric": f"bigmul products/s over the {'quadratic' if kind == 'mulq' else 'NTT'} multiplication sizes "
                  "(u32 limbs, full 2n-limb products), best algorithm per size",
        "value": step_pairs / (step_ms * 1e-3), "unit": "mults/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": step_ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic (seeded splitmix64, uniform limbs)",
        "config": {"workload": "mul_quadratic" if kind == "mulq" else "mul_ntt",
                   "cases": [{"bits": c[0], "pairs": c[1]} for c in cases], "limb_bits": 32,
                   "algorithms": algos, "parallelism": "single-gpu"},
        "roofline": dom.get("roofline"), "per_size": results,
        "cpu_baseline": None if args.no_cpu else cpu_baseline_mul(args, kind, cases),
    }


def graph_replay_timing(ctx, B, A, Bt, out, algo, steps):
    """One call of `algo` captured in a HIP graph (the context's scratch is
    already sized by the eager calls, so nothing allocates while capturing):
    replays, each checked against the eager product with the host's
    synchronisations between them, then `steps` replays back to back, timed
    on the replay stream.  Context for the eager figure: a graph saves the
    host's per-kernel launches, not the GPU's dependent-kernel gaps, and on
    this stack its replays measured about 5 us slower per call than the same
    calls issued back to back."""
    import torch
    stream = torch.cuda.current_stream()
    B.bigmul(ctx, A, Bt, out, algo=algo, stream=stream.cuda_stream)
    torch.cuda.synchronize()
    ref = out.clone()
    g = torch.cuda.CUDAGraph()
    try:
        with torch.cuda.graph(g):
            B.bigmul(ctx, A, Bt, out, algo=algo, stream=torch.cuda.current_stream().cuda_stream)
    except Exception as e:  # a call that cannot be captured is reported, not timed
        torch.cuda.synchronize()
        return {"error": str(e)[:200]}
    checked = 0
    for _ in range(3):
        out.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        if not torch.equal(out, ref):
            return {"error": "replay result differs from the eager product"}
        checked += 1
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        g.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    if not torch.equal(out, ref):
        return {"error": "replay result differs from the eager product"}
    return {"us_per_launch": round(1e3 * e0.elapsed_time(e1) / steps, 2), "replays_checked": checked + 1}


def cpu_baseline_mul(args, kind, cases):
    """The oracle's schoolbook product on the first pairs of each size, one
    task per pair, each size for an equal share of the time budget; products/s
    over the sample."""
    import oracle
    import workloads as W
    oracle.build()
    orc = oracle.get()
    budget = args.cpu_seconds / len(cases)
    pairs, secs, threads, samples = 0, 0.0, 0, []
    for bits, batch in cases:
        cnt = min(batch, 64)
        idx = np.arange(cnt, dtype=np.uint64)
        a, b = W.mul_quad_inputs(bits, pairs=idx) if kind == "mulq" else W.ntt_inputs(bits, batch, pairs=idx)
        t_size, n_size = 0.0, 0
        while t_size < budget:
            t = time.perf_counter()
            orc.mul(a, b)
            t_size += time.perf_counter() - t
            n_size += cnt
            threads = orc.last_threads
        pairs += n_size
        secs += t_size
        samples.append(f"{cnt} pairs x{n_size // cnt} at 2^{bits.bit_length() - 1}")
    # one core: the first 8 pairs of each size, once
    pairs1, secs1, macs1 = 0, 0.0, 0.0
    for bits, batch in cases:
        idx = np.arange(min(batch, 8), dtype=np.uint64)
        a, b = W.mul_quad_inputs(bits, pairs=idx) if kind == "mulq" else W.ntt_inputs(bits, batch, pairs=idx)
        t = time.perf_counter()
        orc.mul(a, b, threads=1)
        secs1 += time.perf_counter() - t
        pairs1 += len(idx)
        macs1 += float(len(idx)) * a.shape[1] ** 2
    return {"value": pairs / secs, "unit": "mults/s", "cores": threads, "kind": "oracle",
            "sample": "first pairs of each size, repeated: " + "; ".join(samples),
            "cpu_model": cpu_info(), "seconds": round(secs, 2),
            "one_core": {"value": pairs1 / secs1, "unit": "mults/s", "cores": 1, "seconds": round(secs1, 2),
                         "u32_macs_per_s": macs1 / secs1, "sample": "first 8 pairs of each size, once"}}


def bench_stream(args):
    """Mixed-size stream: 10^5 pairs, n = max(1, round(2^u / 32)) u32 limbs,
    u ~ U[10, 18], 10 % all-ones, in bursts of log-uniform size in [64, 4096].

    stream path: one bi_stream_submit per burst, in both queue modes: graph
    (descriptor copy + one replay of the captured graph: device binning, one
    persistent list kernel per size class) and host-binned (the copy carries
    the class lists; only the classes present are launched, grids sized to
    their counts).  plain path (baseline): per burst, one uniform bigmul launch per
    size class present, on operands zero-padded to the class's largest size
    (padding prepared before timing).  Both run back to back (saturated), then
    replay one seeded Poisson arrival trace whose offered load is 0.8x the
    plain path's saturated throughput; latency = completion - arrival.
    """
    import torch

    import paper_2405_14642_amd as B
    import workloads as W

    count = args.stream_pairs
    n, ones = W.stream_sizes(count)
    bursts = W.stream_bursts(count)
    bstart = np.concatenate([[0], np.cumsum(bursts)[:-1]]).astype(np.int64)
    a, b, off = W.stream_inputs(np.arange(count), n, ones)
    nn = n.astype(np.int64)
    sum_n2 = float((nn.astype(np.float64) ** 2).sum())
    dA, dB = G.to_dev(a), G.to_dev(b)
    tot = int(nn.sum())
    out = torch.zeros(2 * tot, dtype=torch.int32, device="cuda")
    desc = np.zeros(count, dtype=B.DESC_DTYPE)
    desc["a_off"], desc["b_off"], desc["out_off"], desc["n_limbs"] = off, off, 2 * off, nn
    ctx = B.Context(0)
    tuned = B.autotune(ctx)
    stream = torch.cuda.current_stream()

    # plain path: padded per-(burst, class) operands, built on the device
    cls = np.array([0 if x <= 16 else int(np.ceil(np.log2(x))) - 4 for x in nn], dtype=np.int64)
    off_dev = torch.from_numpy(off.astype(np.int64)).cuda()
    n_dev = torch.from_numpy(nn).cuda()
    zero = torch.zeros(1, dtype=torch.int32, device="cuda")
    flatA = torch.cat([dA.view(torch.int32).reshape(-1), zero])
    flatB = torch.cat([dB.view(torch.int32).reshape(-1), zero])
    plain = []  # per burst: list of (Apad, Bpad, Opad, idx)
    for k in range(len(bursts)):
        sel = np.arange(bstart[k], bstart[k] + bursts[k])
        jobs = []
        for c in np.unique(cls[sel]):
            idx = sel[cls[sel] == c]
            nmax = 16 << int(c)
            it = torch.from_numpy(idx).cuda()
            j = torch.arange(nmax, device="cuda")
            gi = off_dev[it][:, None] + j[None, :]
            valid = j[None, :] < n_dev[it][:, None]
            gi = torch.where(valid, gi, torch.full_like(gi, tot))
            jobs.append((flatA[gi].contiguous(), flatB[gi].contiguous(),
                         torch.empty((len(idx), 2 * nmax), dtype=torch.int32, device="cuda"), idx))
        plain.append(jobs)
    torch.cuda.synchronize()

    def run_plain(k):
        for Ap, Bp, Op, _ in plain[k]:
            B.bigmul(ctx, Ap, Bp, Op, algo=0, stream=stream.cuda_stream)

    q = B.StreamQueue(ctx, dA, dB, out, 32, max_descs=int(bursts.max()), algo=0, use_graph=True)
    qh = B.StreamQueue(ctx, dA, dB, out, 32, max_descs=int(bursts.max()), algo=0, use_graph=False)

    def run_stream(k):
        q.submit(desc[bstart[k]: bstart[k] + bursts[k]])

    def run_host_binned(k):
        qh.submit(desc[bstart[k]: bstart[k] + bursts[k]])

    def saturated(run):
        run(0)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for k in range(len(bursts)):
            run(k)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3

    def replay(run, arrivals):
        torch.cuda.synchronize()
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(len(bursts))]
        e0 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        t0 = time.perf_counter()
        for k in range(len(bursts)):
            while time.perf_counter() - t0 < arrivals[k]:
                pass
            run(k)
            evs[k].record(stream)
        torch.cuda.synchronize()
        lat = np.array([e0.elapsed_time(evs[k]) * 1e-3 - arrivals[k] for k in range(len(bursts))])
        return lat

    modes = (("plain", run_plain), ("stream", run_stream), ("stream_host_binned", run_host_binned))
    sat = {}
    for name, run in modes:
        sat[name] = min(saturated(run) for _ in range(max(1, args.steps // 10 or 1)))
    thr_plain = count / sat["plain"]
    rng = np.random.default_rng(W.DEFAULT_SEED & 0xFFFFFFFF)
    mean_gap = float(bursts.mean()) / (0.8 * thr_plain)
    arrivals = np.concatenate([[0.0], np.cumsum(rng.exponential(mean_gap, len(bursts) - 1))])
    res = {}
    for name, run in modes:
        lat = replay(run, arrivals)
        res[name] = {"saturated_s": round(sat[name], 6), "pairs_per_s": count / sat[name],
                     "sum_n2_per_s": sum_n2 / sat[name],
                     "latency_p50_ms": round(1e3 * float(np.percentile(lat, 50)), 3),
                     "latency_p99_ms": round(1e3 * float(np.percentile(lat, 99)), 3)}
    q.close()
    qh.close()
    best = max(("stream", "stream_host_binned"), key=lambda m: res[m]["pairs_per_s"])

    # cross-check: the stream's results equal the plain per-class launches'
    # (bit-exactness against the oracle is the test suite's job)
    got = out.cpu().numpy().view(np.uint32)
    checked = 0
    for Ap, Bp, Op, idx in plain[len(plain) // 2]:
        Oh = Op.cpu().numpy().view(np.uint32)
        for r, i in enumerate(idx[:8]):
            o, m = int(off[i]), int(nn[i])
            assert (Oh[r, : 2 * m] == got[2 * o: 2 * o + 2 * m]).all(), ("plain result", int(i))
            checked += 1
    # roofline of the mixed stream: the sum over pairs of each product's time
    # at the roofline of its class's tuned algorithm, against the time taken
    ideal_n = {int(m): mul_ideal_seconds(ctx, int(m)) for m in np.unique(nn)}
    ideal = float(sum(ideal_n[int(m)] * c for m, c in zip(*np.unique(nn, return_counts=True))))
    roofline = {"bound": "alu+mfma (per-class tuned algorithm)", "kernel": "whole stream (all class kernels)",
                "achieved": round(sum_n2 / sat[best] / 1e12, 3), "peak": round(sum_n2 / ideal / 1e12, 3),
                "unit": "T u32-MAC-equivalents/s (sum of n^2 per second)", "frac": round(ideal / sat[best], 4),
                "ideal_s": ideal, "traffic": None}
    cpu = None if args.no_cpu else cpu_baseline_stream(args, a, b, off, nn)
    ctx.close()
    return {
        "metric": "products/s over a stream of 10^5 mixed-size multiplications (2^10..2^18 bits, u32 limbs, "
                  "bursts of 64..4096), stream queue, saturated",
        "value": res[best]["pairs_per_s"], "unit": "mults/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": round(1e3 * sat[best], 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic (seeded splitmix64; 10 % all-ones pairs)",
        "config": {"workload": "stream", "pairs": count, "bursts": len(bursts), "limb_bits": 32,
                   "sum_n2": sum_n2, "tuned_algorithm_per_class": tuned, "queue_mode": best,
                   "parallelism": "single-gpu"},
        "stream": res["stream"], "stream_host_binned": res["stream_host_binned"],
        "plain_per_class_launches": res["plain"],
        "speedup_vs_plain": round(sat["plain"] / sat[best], 3), "cross_checked_vs_plain": checked,
        "roofline": roofline, "cpu_baseline": cpu,
    }


def cpu_baseline_stream(args, a, b, off, nn):
    """The oracle over the stream's first pairs, one task per pair, until the
    time budget is spent."""
    import oracle
    oracle.build()
    orc = oracle.get()
    pairs, macs, secs = 0, 0.0, 0.0
    i = 0
    chunk = 256
    while secs < args.cpu_seconds and i < len(nn):
        items = []
        for k in range(i, min(i + chunk, len(nn))):
            o, m = int(off[k]), int(nn[k])
            items.append((a[o: o + m], b[o: o + m]))
        t = time.perf_counter()
        orc.mul_ragged(items)
        secs += time.perf_counter() - t
        pairs += len(items)
        macs += float(sum(len(x) ** 2 for x, _ in items))
        i += chunk
    threads = orc.last_threads
    items = [(a[int(off[k]): int(off[k]) + int(nn[k])], b[int(off[k]): int(off[k]) + int(nn[k])]) for k in range(64)]
    t = time.perf_counter()
    orc.mul_ragged(items, threads=1)
    secs1 = time.perf_counter() - t
    macs1 = float(sum(len(x) ** 2 for x, _ in items))
    return {"value": pairs / secs, "unit": "mults/s", "cores": threads, "kind": "oracle",
            "sample": f"first {pairs} pairs of the stream", "u32_macs_per_s": macs / secs,
            "cpu_model": cpu_info(), "seconds": round(secs, 2),
            "one_core": {"value": 64 / secs1, "unit": "mults/s", "cores": 1, "seconds": round(secs1, 2),
                         "u32_macs_per_s": macs1 / secs1, "sample": "first 64 pairs of the stream, once"}}


def bench_fused(args):
    """The paper's fused programs (Section 6.1) over the addition sweep's
    batches (NumBits x NumInsts = 2^32, u64 limbs): 1-Add (bigadd), 6-Add,
    Poly and the same-length product 1-Mul (Figs. 4-5), one launch each.  6-Add is memory-bound: 3 N/8 bytes per instance
    (two operands in, one result out) against HBM.  Poly is four same-length
    VALU products of n (n + 1) / 2 u32 terms each (n 32-bit words) against the
    VALU multiply-accumulate peak."""
    import torch

    import paper_2405_14642_amd as B
    import workloads as W

    ctx = B.Context(0)
    stream = torch.cuda.current_stream()
    sizes = W.ADD_SWEEP_BITS
    if args.sizes:
        sizes = tuple(int(x) for x in args.sizes.split(","))

    def timed(fn):
        fn()
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        evs = []
        for _ in range(args.steps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            evs.append((e0, e1))
        torch.cuda.synchronize()
        return 1e3 * float(np.mean([x.elapsed_time(y) for x, y in evs]))

    per_size = {}
    add6_s = poly_s = 0.0
    insts = 0
    for bits in sizes:
        a, b = W.add_sweep_inputs(bits)
        n, batch = a.shape[1], a.shape[0]
        A, Bt = G.to_dev(a), G.to_dev(b)
        del a, b
        out = torch.empty_like(A)
        cs = stream.cuda_stream
        us1 = timed(lambda: B.bigadd(ctx, A, Bt, out, None, n_limbs=n, limb_bits=64, batch=batch, stream=cs))
        us6 = timed(lambda: B.fused(ctx, B.PROG_ADD6, A, Bt, out, n_limbs=n, limb_bits=64, batch=batch, stream=cs))
        usp = timed(lambda: B.fused(ctx, B.PROG_POLY, A, Bt, out, n_limbs=n, limb_bits=64, batch=batch, stream=cs))
        usm = timed(lambda: B.fused(ctx, B.PROG_MUL_LOW, A, Bt, out, n_limbs=n, limb_bits=64, batch=batch, stream=cs))
        nbytes = 3 * batch * bits // 8
        n32 = 2 * n
        macs = 4.0 * batch * n32 * (n32 + 1) / 2
        gbs = nbytes / (us6 * 1e-6) / 1e9
        per_size[str(bits)] = {
            "instances": batch, "add1_us": round(us1, 2), "add6_us": round(us6, 2),
            "add6_over_add1": round(us6 / us1, 3), "add6_GB_per_s": round(gbs, 1),
            "add6_hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "poly_us": round(usp, 2),
            "poly_u32_macs_per_s": macs / (usp * 1e-6), "mul_low_us": round(usm, 2),
            "poly_over_mul_low": round(usp / usm, 3),
            "mul_low_roofline": {"bound": "alu", "achieved": round(macs / 4 / (usm * 1e-6) / 1e12, 3),
                                 "peak": round(VALU_MAC_PEAK / 1e12, 3), "unit": "T u32-MAC/s",
                                 "frac": round(macs / 4 / (usm * 1e-6) / VALU_MAC_PEAK, 4)},
            "poly_roofline": {"bound": "alu", "achieved": round(macs / (usp * 1e-6) / 1e12, 3),
                              "peak": round(VALU_MAC_PEAK / 1e12, 3), "unit": "T u32-MAC/s",
                              "frac": round(macs / (usp * 1e-6) / VALU_MAC_PEAK, 4)}}
        add6_s += us6 * 1e-6
        poly_s += usp * 1e-6
        insts += batch
        del A, Bt, out
        torch.cuda.empty_cache()
    ctx.close()
    # dominant 6-Add launch: the slowest one of the sweep (each moves 1.5 GiB)
    dom = max(sizes, key=lambda x: per_size[str(x)]["add6_us"])
    d = per_size[str(dom)]
    cpu = None if args.no_cpu else cpu_baseline_fused(args, W, sizes)
    return {
        "metric": "fused 6-Add programs/s over the 2^10..2^18-bit sweep (u64 limbs, NumBits x NumInsts = 2^32), "
                  "with Poly beside it",
        "value": insts / add6_s, "unit": "programs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * add6_s, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic (seeded splitmix64; 75% uniform, 25% carry-heavy)",
        "config": {"workload": "fused", "sizes_bits": list(sizes), "limb_bits": 64,
                   "programs": ["6-Add", "Poly"], "parallelism": "single-gpu"},
        "roofline": {"bound": "hbm", "kernel": f"fused_add6_kernel at 2^{dom.bit_length() - 1} bits",
                     "achieved": d["add6_GB_per_s"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": d["add6_hbm_frac"], "traffic": None},
        "poly_ms_per_sweep": round(1e3 * poly_s, 3), "per_size": per_size, "cpu_baseline": cpu,
    }


def cpu_baseline_fused(args, W, sizes):
    """The oracle's 6-Add over the first instances of each size, repeated until
    the time budget per size is spent."""
    import oracle
    oracle.build()
    budget = args.cpu_seconds / len(sizes)
    progs, secs = 0, 0.0
    samples = []
    for bits in sizes:
        cnt = max(1, W.add_sweep_pairs(bits) // 16)
        a, b = W.add_sweep_inputs(bits, pairs=np.arange(cnt, dtype=np.uint64))
        t_size, n_size = 0.0, 0
        while t_size < budget:
            t = time.perf_counter()
            oracle.add6(a, b)
            t_size += time.perf_counter() - t
            n_size += cnt
        progs += n_size
        secs += t_size
        samples.append(f"{cnt} instances x{n_size // cnt} at 2^{bits.bit_length() - 1}")
    return {"value": progs / secs, "unit": "programs/s", "cores": oracle.get().last_threads, "kind": "oracle",
            "sample": "first sixteenth of each size's batch, repeated: " + "; ".join(samples),
            "cpu_model": cpu_info(), "seconds": round(secs, 2)}


def bench_copy(args):
    """A plain device-to-device copy of 1 GiB (torch's copy kernel): the
    reference of known size for the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = 1 << 28
    src = torch.ones(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        dst.copy_(src)
    torch.cuda.synchronize()
    evs = []
    for _ in range(args.steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        dst.copy_(src)
        e1.record(stream)
        evs.append((e0, e1))
    torch.cuda.synchronize()
    us = 1e3 * float(np.mean([x.elapsed_time(y) for x, y in evs]))
    nbytes = 4 * n
    return {"metric": "device copy bandwidth (read + write)", "value": 2 * nbytes / (us * 1e-6) / 1e9,
            "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": us / 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "int32", "data": "synthetic (constant)",
            "config": {"workload": "copy", "bytes_read": nbytes, "bytes_written": nbytes,
                       "parallelism": "single-gpu"},
            "roofline": {"bound": "hbm", "achieved": round(2 * nbytes / (us * 1e-6) / 1e9, 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(2 * nbytes / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4), "traffic": None},
            "cpu_baseline": None}


def bench_add_large(args):
    """One integer pair per size, 2^20..2^34 bits (u32 limbs), added by
    bigadd_large (tile pass, summary scan, carry fix-up: one call).  Uniform
    operands, and the ripple pattern (a = all-ones, b = 1), whose carry
    crosses every limb so the fix-up rewrites the whole sum."""
    import torch

    import paper_2405_14642_amd as B
    import workloads as W

    ctx = B.Context(0)
    stream = torch.cuda.current_stream()
    sizes = W.LARGE_ADD_BITS
    if args.sizes:
        sizes = tuple(int(x) for x in args.sizes.split(","))
    per_size = {}
    main_bits = 1 << 32
    step_ms = 0.0
    for bits in sizes:
        n = bits // 32
        for pattern in ("uniform", "ripple"):
            a, b = W.large_add_inputs(n, pattern)
            A, Bt = G.to_dev(a), G.to_dev(b)
            del a, b
            out = torch.empty_like(A)
            carry = torch.empty(1, dtype=torch.uint8, device="cuda")

            def launch():
                B.bigadd_large(ctx, A, Bt, out, carry, stream=stream.cuda_stream)

            for _ in range(args.warmup):
                launch()
            torch.cuda.synchronize()
            evs = []
            for _ in range(args.steps):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                launch()
                e1.record(stream)
                evs.append((e0, e1))
            torch.cuda.synchronize()
            us = 1e3 * float(np.mean([x.elapsed_time(y) for x, y in evs]))
            nbytes = 12 * n  # read a and b, write the sum
            gbs = nbytes / (us * 1e-6) / 1e9
            per_size.setdefault(str(bits), {})[pattern] = {
                "us_per_call": round(us, 2), "GB_per_s": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                "adds_per_s": 1e6 / us}
            if pattern == "uniform":
                step_ms += us / 1e3
            del A, Bt, out
            torch.cuda.empty_cache()
    ctx.close()
    key = str(main_bits) if str(main_bits) in per_size else str(sizes[-1])
    main = per_size[key]["uniform"]
    nb = 12 * (int(key) // 32)
    case = f"2^{int(key).bit_length() - 1} bits uniform"
    roofline = {"bound": "hbm", "kernel": "bigadd_large call (large_add_tile_kernel + scan + fix-up + walk)",
                "achieved": main["GB_per_s"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(main["GB_per_s"] / HBM_PEAK_GBS, 4), "traffic": measured_large_traffic(case),
                "traffic_source": "profiles/bigadd_large_traffic.md",
                "avg_launch_us": main["us_per_call"], "algorithmic_bytes_per_launch": nb}
    cpu = None if args.no_cpu else cpu_baseline_add_large(args, W, int(key))
    return {
        "metric": f"bigadd_large additions/s of one 2^{int(key).bit_length() - 1}-bit integer pair (u32 limbs)",
        "value": main["adds_per_s"], "unit": "adds/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": step_ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic (seeded splitmix64, uniform; ripple = all-ones + 1)",
        "config": {"workload": "add_large", "sizes_bits": list(sizes), "limb_bits": 32,
                   "parallelism": "single-gpu"},
        "roofline": roofline, "per_size": per_size, "cpu_baseline": cpu,
    }


def large_ntt_block_words(n32):
    """Block size (words) bigmul_large's NTT path picks by default, as the
    library reports it."""
    import paper_2405_14642_amd as B
    return B.mul_large_plan(n32, 32, 0)[0] // 32


def large_ntt_butterflies(n32, bw):
    """Radix-2 butterflies of one bigmul_large product on the NTT path, both
    primes: per block 2 forward row transforms, 2k - 1 inverse rows, and per
    row position the column transforms (4 forward and 2 inverse halves of H
    points)."""
    k = -(-n32 // bw)
    m = 11
    while (1 << m) < 4 * bw:
        m += 1
    L = 1 << m
    r = 0
    while (2 << r) < 2 * k - 1:
        r += 1
    H = 1 << r
    rows = (2 * k + 2 * k - 1) * (L // 2) * m
    cols = L * 6 * (H // 2) * r
    return 2.0 * (rows + cols), k, L, H


def bench_mul_large(args):
    """One pair per size, 2^19..2^24 bits (u32 limbs, uniform), multiplied by
    bigmul_large: the default NTT path is a two-dimensional convolution (row
    transforms per block, column transforms across blocks, CRT, a fold and
    the multi-workgroup addition); its roofline counts the butterflies of
    those transforms against the butterfly peak.  Beside it: other block
    sizes, and the k^2 block products forced to the int8-MFMA schoolbook."""
    import torch

    import paper_2405_14642_amd as B
    import workloads as W

    ctx = B.Context(0)
    stream = torch.cuda.current_stream()
    sizes = (1 << 19, 1 << 20, 1 << 22, 1 << 24)
    if args.sizes:
        sizes = tuple(int(x) for x in args.sizes.split(","))
    per_size = {}
    step_ms = 0.0
    for bits in sizes:
        n = bits // 32
        a, b = W.large_add_inputs(n)
        A, Bt = G.to_dev(a), G.to_dev(b)
        out = G.empty_dev(2 * n, np.uint32)

        def timed(algo, block_bits=0):
            for _ in range(args.warmup + 1):
                B.bigmul_large(ctx, A, Bt, out, algo=algo, block_bits=block_bits, stream=stream.cuda_stream)
            torch.cuda.synchronize()
            evs = []
            for _ in range(args.steps):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                B.bigmul_large(ctx, A, Bt, out, algo=algo, block_bits=block_bits, stream=stream.cuda_stream)
                e1.record(stream)
                evs.append((e0, e1))
            torch.cuda.synchronize()
            return 1e3 * float(np.mean([x.elapsed_time(y) for x, y in evs]))

        us = timed(B.MUL_AUTO)
        bw = large_ntt_block_words(n)
        bfly, k, L, H = large_ntt_butterflies(n, bw)
        roof = {"bound": "alu", "achieved": round(bfly / (us * 1e-6) / 1e12, 3),
                "peak": round(NTT_BFLY_PEAK / 1e12, 3), "unit": "T butterflies/s",
                "frac": round(bfly / (us * 1e-6) / NTT_BFLY_PEAK, 4), "butterflies_per_call": bfly}
        by_block = {}
        for bb in (1 << 14, 1 << 15, 1 << 16, 1 << 17, 1 << 18):
            if -(-n // (bb // 32)) <= 64:
                by_block[str(bb)] = round(timed(B.MUL_AUTO, bb), 2)
        mfma_blocks = None
        if bits <= (1 << 22):  # k^2 block products grow quadratically
            mfma_blocks = round(timed(B.MUL_SCHOOL_MFMA), 2)
        per_size[str(bits)] = {"us_per_call": round(us, 2), "block_bits": 32 * bw, "blocks": k,
                               "row_length": L, "column_half_length": H, "mults_per_s": 1e6 / us, "roofline": roof,
                               "us_per_call_by_block_bits": by_block,
                               "us_per_call_mfma_block_products": mfma_blocks}
        step_ms += us / 1e3
        del A, Bt, out
    ctx.close()
    key = str(1 << 24) if str(1 << 24) in per_size else str(sizes[-1])
    main = per_size[key]
    return {
        "metric": f"bigmul_large products/s of one 2^{int(key).bit_length() - 1}-bit pair (u32 limbs)",
        "value": main["mults_per_s"], "unit": "mults/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": step_ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic (seeded splitmix64, uniform)",
        "config": {"workload": "mul_large", "sizes_bits": list(sizes), "limb_bits": 32, "parallelism": "single-gpu"},
        "roofline": dict(main["roofline"], traffic=None),
        "per_size": per_size, "cpu_baseline": None,
    }


def cpu_baseline_add_large(args, W, bits):
    import oracle
    oracle.build()
    orc = oracle.get()
    a, b = W.large_add_inputs(bits // 32)
    a, b = a[None, :], b[None, :]
    reps, secs = 0, 0.0
    while secs < args.cpu_seconds:
        t = time.perf_counter()
        orc.add(a, b)
        secs += time.perf_counter() - t
        reps += 1
    # The oracle parallelises over instances: one instance keeps one thread busy.
    return {"value": reps / secs, "unit": "adds/s", "cores": min(orc.last_threads, 1), "kind": "oracle",
            "sample": f"the uniform 2^{bits.bit_length() - 1}-bit pair, {reps} additions",
            "cpu_model": cpu_info(), "seconds": round(secs, 2)}


def cpu_baseline_add(args, W):
    import oracle
    oracle.build()
    orc = oracle.get()
    budget = args.cpu_seconds / len(W.ADD_SWEEP_BITS)
    adds, secs, threads = 0, 0.0, 0
    samples = []
    for bits in W.ADD_SWEEP_BITS:
        total = W.add_sweep_pairs(bits)
        cnt = max(1, total // 4)
        a, b = W.add_sweep_inputs(bits, pairs=np.arange(cnt, dtype=np.uint64))
        t_size, n_size = 0.0, 0
        while t_size < budget:
            t = time.perf_counter()
            orc.add(a, b)
            t_size += time.perf_counter() - t
            n_size += cnt
            threads = orc.last_threads
        adds += n_size
        secs += t_size
        samples.append(f"{cnt} pairs x{n_size // cnt} at 2^{bits.bit_length() - 1}")
    # one core: the first 1/16 of each size's sample, once
    adds1, secs1 = 0, 0.0
    for bits in W.ADD_SWEEP_BITS:
        cnt = max(1, W.add_sweep_pairs(bits) // 64)
        a, b = W.add_sweep_inputs(bits, pairs=np.arange(cnt, dtype=np.uint64))
        t = time.perf_counter()
        orc.add(a, b, threads=1)
        secs1 += time.perf_counter() - t
        adds1 += cnt
    return {"value": adds / secs, "unit": "adds/s", "cores": threads, "kind": "oracle",
            "sample": "first quarter of each size's batch, repeated: " + "; ".join(samples),
            "cpu_model": cpu_info(), "seconds": round(secs, 2),
            "one_core": {"value": adds1 / secs1, "unit": "adds/s", "cores": 1, "seconds": round(secs1, 2),
                         "sample": "first 1/64 of each size's batch, once"}}


# Issue-rate probe kinds (libbiprobe.so): instruction measured and what one
# "op" is.
PROBE_KINDS = (
    (0, "v_add_u32", "lane-op"),
    (1, "v_addc_co_u32 (VOP3, carry in SGPR pair)", "lane-op"),
    (2, "v_mad_u64_u32", "lane-op"),
    (3, "v_mul_lo_u32", "lane-op"),
    (4, "v_mul_hi_u32", "lane-op"),
    (5, "v_mfma_i32_32x32x32_i8", "int8 MAC"),
    (6, "schoolbook term: v_mad_u64_u32 + v_addc_co_u32", "term"),
)
SIMDS = 256 * 4          # 256 CUs x 4 SIMDs
CLOCK_PEAK_HZ = 2.4e9    # MI355X peak engine clock


def bench_peaks(args):
    """Register-resident issue rates of the instructions the integer-op
    rooflines count, with the shader clock each loop ran at (s_memtime
    against the 100 MHz s_memrealtime); per kind the best of 1, 2, 4 and 8
    waves per SIMD.  ops/clk/SIMD = rate / (1024 SIMDs x measured clock)."""
    import ctypes
    import torch
    torch.cuda.init()
    torch.zeros(1, device="cuda")
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2405_14642_amd", "libbiprobe.so"))
    D = ctypes.c_double
    lib.bi_probe_rate.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(D), ctypes.POINTER(D),
                                  ctypes.POINTER(D)]
    lib.bi_probe_rate.restype = ctypes.c_int
    rates = {}
    for kind, name, unit in PROBE_KINDS:
        best = None
        for waves in (1, 2, 4, 8):
            ops, clk, sec = D(), D(), D()
            iters = 4000 if kind == 5 else 20000
            st = lib.bi_probe_rate(kind, iters, waves, ctypes.byref(ops), ctypes.byref(clk), ctypes.byref(sec))
            if st != 0:
                raise RuntimeError(f"probe {name} failed with HIP error {st}")
            if best is None or ops.value > best[0]:
                best = (ops.value, clk.value, sec.value, waves)
        ops, clk, sec, waves = best
        per_clk = ops / (SIMDS * clk) if clk else None
        rates[name] = {"unit": unit + "/s", "rate": ops, "clock_hz": round(clk), "seconds": round(sec, 6),
                       "waves_per_simd": waves, "per_clk_per_simd": round(per_clk, 3) if per_clk else None,
                       "at_2p4GHz": per_clk * SIMDS * CLOCK_PEAK_HZ if per_clk else None}
    return {"metric": "register-resident issue rates (ops/s) of the instructions the integer-op rooflines count",
            "value": rates["v_mad_u64_u32"]["rate"], "unit": "v_mad_u64_u32 lane-ops/s", "n_gpus": 1,
            "steps": 1, "warmup": 1, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "u32", "data": "synthetic (register-resident loops)",
            "config": {"workload": "peaks", "parallelism": "single-gpu"}, "rates": rates,
            "roofline": None, "cpu_baseline": None}


SUB_KEYS = ("metric", "value", "unit", "ms_per_step", "dtype", "config", "roofline", "per_size", "cpu_baseline")


def bench_all(args):
    """The default run: the addition sweep (the headline value: additions/s,
    HBM roofline), then the quadratic and NTT multiplication sizes (every
    algorithm, best per size, integer-op rooflines) and the mixed-size
    stream, each carried in the one JSON line with its own roofline and CPU
    baseline."""
    import torch
    res = bench_add(args)
    torch.cuda.empty_cache()
    for key, kind in (("mul_quadratic", "mulq"), ("mul_ntt", "ntt")):
        sub = bench_mul(args, kind)
        res[key] = {k: sub[k] for k in SUB_KEYS}
        torch.cuda.empty_cache()
    sub = bench_stream(args)
    res["stream"] = {k: v for k, v in sub.items() if k not in ("n_gpus", "steps", "warmup", "higher_is_better",
                                                                  "scaling", "vs_baseline", "data")}
    torch.cuda.empty_cache()
    res["metric"] = ("integer adds/s and mults/s per size (2^10..2^18 bits) with % of the HBM / integer-op "
                     "roofline; value: additions/s over the 2^10..2^18-bit sweep (u64 limbs, 1 GiB of operands "
                     "per size)")
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the batch shards by instance "
                          "across GPUs with no exchange, so --gpus N > 1 is not supported"}))
        sys.exit(2)
    if args.workload == "all":
        res = bench_all(args)
    elif args.workload == "add":
        res = bench_add(args)
    elif args.workload == "add_large":
        res = bench_add_large(args)
    elif args.workload == "mul_large":
        res = bench_mul_large(args)
    elif args.workload == "stream":
        res = bench_stream(args)
    elif args.workload == "peaks":
        res = bench_peaks(args)
    elif args.workload == "copy":
        res = bench_copy(args)
    elif args.workload == "fused":
        res = bench_fused(args)
    else:
        res = bench_mul(args, args.workload)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
