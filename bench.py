"""Benchmark of the batched big-integer hot path on one MI355X.

Default workload: the addition bandwidth sweep.  One step adds, at each of
2^10, 2^12, 2^14, 2^16 and 2^18 bits (u64 limbs), a batch of 2^32/N pairs
(1 GiB of operands, 0.5 GiB of sums per size), i.e. five bigadd launches.
Inputs are generated on the host (seeded, 75 % uniform, 25 % carry-heavy),
copied to HBM once, and stay resident; the timed region contains only the
kernels.  Every launch is timed with HIP events on the stream it runs on.

Other workloads (--workload): mulq (quadratic multiplication sizes),
ntt (NTT-multiplication sizes); each prints its own JSON line.

Prints one JSON line (rank 0, one GPU):
  value   whole-job additions per second over the step (all five sizes);
  roofline   for the dominant kernel: algorithmic bytes per launch (3 N/8 per
             pair = 1.5 GiB) over its average launch time, against 8 TB/s;
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


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="add", choices=["add", "mulq", "ntt"])
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    p.add_argument("--cpu-seconds", type=float, default=12.0, help="CPU baseline budget")
    p.add_argument("--sizes", default="", help="comma-separated subset of sizes in bits (profiling runs)")
    p.add_argument("--algos", default="valu,mfma,ntt", help="multiplication algorithms to time")
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
    from tests import gpu_util as G

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
    roofline = {"bound": "hbm", "kernel": add_kernel_name(dom_bits // 64, 64) + f" at 2^{dom_bits.bit_length() - 1} bits",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
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


# Peak rates used for the multiplication rooflines, derived from the unit counts and clock:
# VALU schoolbook: one v_mad_u64_u32 (16 lanes/clk/SIMD) + one v_addc_co_u32
# (32 lanes/clk/SIMD) per 32x32-bit product term -> 10.67 terms/clk/SIMD,
# x 1024 SIMDs x 2.4 GHz.
VALU_MAC_PEAK = 1024 * (16 * 32 / 48) * 2.4e9   # 2.62e13 u32 MAC/s
# NTT: a radix-2 butterfly with a Shoup twiddle is 3 multiply-class
# (16 lanes/clk/SIMD) + 7 add-class (32 lanes/clk/SIMD) instructions.
NTT_BFLY_PEAK = 1024 * 2.4e9 / (3 / 16 + 7 / 32)  # 6.05e12 butterflies/s
MFMA_I8_PEAK_OPS = 5.0e15                        # dense int8, ops (2 per MAC)

ALGO_IDS = {"valu": 1, "mfma": 2, "ntt": 3}


def bench_mul(args, kind):
    import torch

    import paper_2405_14642_amd as B
    import workloads as W
    from tests import gpu_util as G

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
            evs = []
            for _ in range(args.steps):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                B.bigmul(ctx, A, Bt, out, algo=algo, stream=stream.cuda_stream)
                e1.record(stream)
                evs.append((e0, e1))
            torch.cuda.synchronize()
            us = 1e3 * float(np.mean([x.elapsed_time(y) for x, y in evs]))
            macs = float(batch) * n * n
            r = {"us_per_launch": round(us, 2), "mults_per_s": batch / (us * 1e-6),
                 "u32_macs_per_s": macs / (us * 1e-6)}
            if name == "valu":
                r["roofline"] = {"bound": "alu", "achieved": round(macs / (us * 1e-6) / 1e12, 3),
                                 "peak": round(VALU_MAC_PEAK / 1e12, 3), "unit": "T u32-MAC/s",
                                 "frac": round(macs / (us * 1e-6) / VALU_MAC_PEAK, 4)}
            elif name == "ntt":
                m = 11
                while (1 << m) < 4 * n:
                    m += 1
                bfly = 2.0 * 3 * batch * (1 << m) / 2 * m
                r["butterflies_per_launch"] = bfly
                r["roofline"] = {"bound": "alu", "achieved": round(bfly / (us * 1e-6) / 1e12, 3),
                                 "peak": round(NTT_BFLY_PEAK / 1e12, 3), "unit": "T butterflies/s",
                                 "frac": round(bfly / (us * 1e-6) / NTT_BFLY_PEAK, 4)}
            elif name == "mfma":
                ops = 2.0 * batch * (4 * n) ** 2
                r["roofline"] = {"bound": "mfma", "achieved": round(ops / (us * 1e-6) / 1e12, 1),
                                 "peak": MFMA_I8_PEAK_OPS / 1e12, "unit": "TOP/s (int8)",
                                 "frac": round(ops / (us * 1e-6) / MFMA_I8_PEAK_OPS, 4)}
            results.setdefault(str(bits), {})[name] = r
            if best is None or us < best[1]:
                best = (name, us)
        if best:
            results[str(bits)]["best"] = best[0]
            step_ms += best[1] / 1e3
            step_pairs += batch
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
        "roofline": dom.get("roofline"), "per_size": results, "cpu_baseline": None,
    }


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
    return {"value": adds / secs, "unit": "adds/s", "cores": threads, "kind": "oracle",
            "sample": "first quarter of each size's batch, repeated: " + "; ".join(samples),
            "cpu_model": cpu_info(), "seconds": round(secs, 2)}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the batch shards by instance "
                          "across GPUs with no exchange, so --gpus N > 1 is not supported"}))
        sys.exit(2)
    if args.workload == "add":
        res = bench_add(args)
    else:
        res = bench_mul(args, args.workload)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
