// On-device autotuning: per ragged size class it first picks the VALU
// schoolbook's schedule (output words per lane Q = 2 or 4, the paper's
// sequentialisation factor, and waves per workgroup), then times every
// multiplication algorithm on synthetic operands of the class's largest size
// and keeps the fastest (used by BI_MUL_AUTO and bigmul_v); it also picks the
// addition schedule for instances of 2, 3-4 and 5-8 rows.  The paper tunes code-version thresholds the same way
// (Section 5.1, Futhark's autotuned thresholds); here the choices are the
// kernel families and their schedules.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "bi_internal.hpp"

namespace bi {

__global__ void fill_hash_kernel(uint32_t *p, uint64_t n, uint32_t seed) {
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x) {
        uint32_t x = uint32_t(i) ^ seed ^ uint32_t(i >> 32) * 0x9E3779B9u;
        x ^= x >> 16; x *= 0x7FEB352Du; x ^= x >> 15; x *= 0x846CA68Bu; x ^= x >> 16;
        p[i] = x;
    }
}

namespace {

struct Timer {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    Timer() {
        (void)hipEventCreate(&e0);
        (void)hipEventCreate(&e1);
    }
    ~Timer() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

template <class F>
bi_status time_us(hipStream_t st, Timer &t, int reps, F &&launch, float *us) {
    bi_status s = launch();  // warm-up (also first-use attribute set-up)
    if (s != BI_OK) return s;
    if (hipEventRecord(t.e0, st) != hipSuccess) return BI_EHIP;
    for (int r = 0; r < reps; ++r)
        if ((s = launch()) != BI_OK) return s;
    if (hipEventRecord(t.e1, st) != hipSuccess || hipEventSynchronize(t.e1) != hipSuccess) return BI_EHIP;
    float ms = 0;
    if (hipEventElapsedTime(&ms, t.e0, t.e1) != hipSuccess) return BI_EHIP;
    *us = 1000.0f * ms / reps;
    return BI_OK;
}

constexpr uint64_t kRaggedMax = 4096;  // instances of a ragged timing batch
const int kAlgos[5] = {BI_MUL_SCHOOL_VALU, BI_MUL_SCHOOL_MFMA, BI_MUL_NTT, BI_MUL_NTT_PF64, BI_MUL_KARATSUBA};

// The list algorithm of class k from a ragged batch: instances of sizes
// spread log-uniformly over the class (a fixed 64-bit LCG), operands at a +
// i nmax and b + i nmax, results at o + 2 i nmax, launched as the one class
// of a host-binned batch; every algorithm that runs the class is timed and
// the fastest kept in c.tune.list_algo[k].
bi_status tune_ragged_class(Ctx &c, uint32_t k, const uint32_t *a, const uint32_t *b, uint32_t *o, uint64_t limbs,
                            void *rdesc, hipStream_t st, Timer &tm) {
    const uint32_t nmax = class_nmax(k), nmin = k ? nmax / 2 + 1 : 1;
    const uint64_t count = std::min<uint64_t>(limbs / nmax, kRaggedMax);
    std::vector<bi_desc> d(count);
    std::vector<uint32_t> list(count);
    uint64_t x = 0x2405146420ull + k;
    for (uint64_t i = 0; i < count; ++i) {
        x = x * 6364136223846793005ull + 1442695040888963407ull;
        const double u = double(x >> 11) * (1.0 / 9007199254740992.0);  // [0, 1)
        uint32_t n = uint32_t(double(nmin) * std::pow(double(nmax) / double(nmin), u));
        n = std::min(std::max(n, nmin), nmax);
        d[i] = bi_desc{i * nmax, i * nmax, 2 * i * nmax, n, 0};
        list[i] = uint32_t(i);
    }
    auto *dd = static_cast<bi_desc *>(rdesc);
    auto *dl = reinterpret_cast<uint32_t *>(dd + kRaggedMax);
    auto *dc = dl + kRaggedMax;
    uint32_t hc[kNumClasses] = {};
    hc[k] = uint32_t(count);
    if (hipMemcpyAsync(dd, d.data(), count * sizeof(bi_desc), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(dl, list.data(), count * sizeof(uint32_t), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(dc, hc, sizeof hc, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return set_error(BI_EHIP, "autotune descriptor copy");
    void *scr = nullptr;
    bi_status s = ctx_scratch(c, batch_scratch_bytes(count, c.num_cus), st, &scr);
    if (s != BI_OK) return s;
    float best = 0;
    int best_algo = c.tune.list_algo[k];
    for (int al : kAlgos) {
        if (!algo_supports(al, nmax)) continue;
        float us = 0;
        s = time_us(st, tm, 3, [&]() {
            return launch_bigmul_v_binned(c, c.tune, a, b, o, dd, dl, dc, hc, 32, al, scr, st) == hipSuccess ? BI_OK
                                                                                                          : BI_EHIP;
        }, &us);
        if (s != BI_OK) return s;
        if (best == 0 || us < best) {
            best = us;
            best_algo = al;
        }
    }
    c.tune.list_algo[k] = best_algo;
    return BI_OK;
}

}  // namespace

bi_status autotune(Ctx &c, hipStream_t st, int *algo_out, uint32_t n_out) {
    // Operand space: 2^22 32-bit limbs per operand (16 MiB), products 2x.
    const uint64_t limbs = uint64_t(1) << 22;
    uint32_t *buf = nullptr;
    if (hipMalloc(&buf, 4 * limbs * sizeof(uint32_t)) != hipSuccess) return set_error(BI_ENOMEM, "autotune buffers");
    uint32_t *a = buf, *b = buf + limbs, *o = buf + 2 * limbs;
    hipLaunchKernelGGL(fill_hash_kernel, dim3(1024), dim3(256), 0, st, a, 2 * limbs, 0x2405u);
    Timer tm;
    bi_status s = BI_OK;
    // descriptors, list and count of the ragged batches
    void *rdesc = nullptr;
    if (hipMalloc(&rdesc, kRaggedMax * (sizeof(bi_desc) + sizeof(uint32_t)) + 256) != hipSuccess) {
        (void)hipFree(buf);
        return set_error(BI_ENOMEM, "autotune buffers");
    }
    const int algos[5] = {BI_MUL_SCHOOL_VALU, BI_MUL_SCHOOL_MFMA, BI_MUL_NTT, BI_MUL_NTT_PF64, BI_MUL_KARATSUBA};
    for (uint32_t k = 0; k < kNumClasses && s == BI_OK; ++k) {
        const uint32_t n = class_nmax(k);
        uint64_t batch = limbs / n;
        if (batch > 65536) batch = 65536;
        // VALU schedule: every (Q, waves) whose LDS fits, fastest kept
        {
            float best_v = 0;
            uint8_t bq = 0, bw = 0;
            for (int Q : {2, 4}) {
                for (int NW : {1, 2, 4, 8, 16}) {
                    if (!valu_plan_fits(n, Q, NW, nullptr)) continue;
                    c.tune.valu_q[k] = uint8_t(Q);
                    c.tune.valu_nw[k] = uint8_t(NW);
                    float us = 0;
                    s = time_us(st, tm, 3, [&]() { return dispatch_bigmul(c, a, b, o, n, batch, BI_MUL_SCHOOL_VALU, st); },
                                &us);
                    if (s != BI_OK) break;
                    if (best_v == 0 || us < best_v) {
                        best_v = us;
                        bq = uint8_t(Q);
                        bw = uint8_t(NW);
                    }
                }
                if (s != BI_OK) break;
            }
            c.tune.valu_q[k] = bq;
            c.tune.valu_nw[k] = bw;
            if (s != BI_OK) break;
        }
        float best = 0;
        int best_algo = c.tune.mul_algo[k];
        for (int al : algos) {
            if (!algo_supports(al, n)) continue;
            // Karatsuba: each base size that gives a different level count;
            // the class keeps the fastest base (whichever algorithm wins)
            int last_levels = -1;
            float kbest = 0;
            uint16_t kbase = c.tune.kara_base[k];
            for (uint32_t base : kKaraBases) {
                if (al != BI_MUL_KARATSUBA && base != kKaraBases[0]) break;
                if (al == BI_MUL_KARATSUBA) {
                    const int lv = kara_plan(n, base).levels;
                    if (lv == last_levels) continue;
                    last_levels = lv;
                    c.tune.kara_base[k] = uint16_t(base);
                }
                float us = 0;
                s = time_us(st, tm, 3, [&]() { return dispatch_bigmul(c, a, b, o, n, batch, al, st); }, &us);
                if (s != BI_OK) break;
                if (al == BI_MUL_KARATSUBA && (kbest == 0 || us < kbest)) {
                    kbest = us;
                    kbase = uint16_t(base);
                }
                if (best == 0 || us < best) {
                    best = us;
                    best_algo = al;
                }
            }
            if (al == BI_MUL_KARATSUBA) c.tune.kara_base[k] = kbase;
            if (s != BI_OK) break;
        }
        c.tune.mul_algo[k] = best_algo;
        if (s != BI_OK) break;
        s = tune_ragged_class(c, k, a, b, o, limbs, rdesc, st, tm);
    }
    if (rdesc) (void)hipFree(rdesc);
    // Addition: workgroup-cooperative vs one wave per instance, per row class.
    for (int rc = 0; rc < 3 && s == BI_OK; ++rc) {
        const uint32_t rows = rc == 0 ? 2 : rc == 1 ? 4 : 8;
        const uint64_t inst_bytes = uint64_t(rows) * 64 * 16;
        const uint64_t batch = (limbs * 4) / inst_bytes;
        float t_coop = 0, t_multi = 0;
        AddTune t = c.add;
        for (int multi = 0; multi < 2 && s == BI_OK; ++multi) {
            if (rc == 0) t.multi2 = multi; else if (rc == 1) t.multi4 = multi; else t.multi8 = multi;
            float us = 0;
            s = time_us(st, tm, 5, [&]() {
                return launch_bigadd(a, b, o, nullptr, inst_bytes, batch, st, t) == hipSuccess ? BI_OK : BI_EHIP;
            }, &us);
            (multi ? t_multi : t_coop) = us;
        }
        const bool m = s == BI_OK && t_multi < t_coop;
        if (rc == 0) c.add.multi2 = m; else if (rc == 1) c.add.multi4 = m; else c.add.multi8 = m;
    }
    (void)hipStreamSynchronize(st);
    (void)hipFree(buf);
    if (s != BI_OK) return s;
    if (algo_out)
        for (uint32_t k = 0; k < n_out && k < kNumClasses; ++k) algo_out[k] = c.tune.mul_algo[k];
    return BI_OK;
}

// File format (text, one record per line):
//   bigint-tune 1
//   arch <gcnArchName>
//   hip <runtime version>
//   mul_algo <10 algorithm ids>
//   valu_q <10 values>    valu_nw <10 values>
//   add_multi <multi2> <multi4> <multi8>
//   kara_base <10 values>   list_algo <10 algorithm ids>
//   (version 2; a version-1 file gives the default Karatsuba bases and its
//   mul_algo table to ragged batches as well)
bi_status tune_save(const Ctx &c, const char *path) {
    std::FILE *f = std::fopen(path, "w");
    if (!f) return set_error(BI_EINVAL, "cannot open %s for writing", path);
    std::fprintf(f, "bigint-tune 2\narch %s\nhip %d\nmul_algo", c.arch, c.hip_version);
    for (uint32_t k = 0; k < kNumClasses; ++k) std::fprintf(f, " %d", c.tune.mul_algo[k]);
    std::fprintf(f, "\nvalu_q");
    for (uint32_t k = 0; k < kNumClasses; ++k) std::fprintf(f, " %d", int(c.tune.valu_q[k]));
    std::fprintf(f, "\nvalu_nw");
    for (uint32_t k = 0; k < kNumClasses; ++k) std::fprintf(f, " %d", int(c.tune.valu_nw[k]));
    std::fprintf(f, "\nadd_multi %d %d %d\nkara_base", int(c.add.multi2), int(c.add.multi4), int(c.add.multi8));
    for (uint32_t k = 0; k < kNumClasses; ++k) std::fprintf(f, " %d", int(c.tune.kara_base[k]));
    std::fprintf(f, "\nlist_algo");
    for (uint32_t k = 0; k < kNumClasses; ++k) std::fprintf(f, " %d", c.tune.list_algo[k]);
    std::fprintf(f, "\n");
    const bool ok = std::fclose(f) == 0;
    return ok ? BI_OK : set_error(BI_EINVAL, "writing %s failed", path);
}

bi_status tune_load(Ctx &c, const char *path) {
    std::FILE *f = std::fopen(path, "r");
    if (!f) return set_error(BI_EINVAL, "cannot open %s", path);
    char arch[64] = {}, key[32] = {};
    int version = -1, hip = 0;
    int algo[kNumClasses], q[kNumClasses], nw[kNumClasses], m[3], kb[kNumClasses], la[kNumClasses];
    // each record opens with its key, compared as a whole token
    auto expect = [&](const char *k) { return std::fscanf(f, "%31s", key) == 1 && std::strcmp(key, k) == 0; };
    auto ints = [&](int *v, uint32_t cnt) {
        for (uint32_t i = 0; i < cnt; ++i)
            if (std::fscanf(f, "%d", &v[i]) != 1) return false;
        return true;
    };
    bool ok = expect("bigint-tune") && ints(&version, 1) && (version == 1 || version == 2) && expect("arch") &&
              std::fscanf(f, "%63s", arch) == 1 && expect("hip") && ints(&hip, 1) && expect("mul_algo") &&
              ints(algo, kNumClasses) && expect("valu_q") && ints(q, kNumClasses) && expect("valu_nw") &&
              ints(nw, kNumClasses) && expect("add_multi") && ints(m, 3);
    for (uint32_t k = 0; k < kNumClasses; ++k) {  // version 1: ragged batches used the uniform table
        kb[k] = int(kKaraBase);
        la[k] = algo[k];
    }
    if (ok && version == 2) ok = expect("kara_base") && ints(kb, kNumClasses) && expect("list_algo") && ints(la, kNumClasses);
    std::fclose(f);
    if (!ok) return set_error(BI_EINVAL, "%s is not a tuning file", path);
    if (std::strcmp(arch, c.arch) != 0 || hip != c.hip_version)
        return set_error(BI_EINVAL, "%s was tuned for %s with HIP %d, this context is %s with HIP %d", path, arch, hip,
                         c.arch, c.hip_version);
    for (uint32_t k = 0; k < kNumClasses; ++k) {
        if (!algo_supports(algo[k], class_nmax(k)) || !algo_supports(la[k], class_nmax(k)))
            return set_error(BI_EINVAL, "%s: algorithm %d / %d cannot run size class %u", path, algo[k], la[k], k);
        if (!(q[k] == 0 && nw[k] == 0) && !valu_plan_fits(class_nmax(k), q[k], nw[k], nullptr))
            return set_error(BI_EINVAL, "%s: VALU schedule (%d, %d) does not fit size class %u", path, q[k], nw[k], k);
        if (!kara_base_valid(uint32_t(kb[k])))
            return set_error(BI_EINVAL, "%s: Karatsuba base %d of size class %u is not one of 512, 1024, 2048", path,
                             kb[k], k);
    }
    for (uint32_t k = 0; k < kNumClasses; ++k) {
        c.tune.mul_algo[k] = algo[k];
        c.tune.valu_q[k] = uint8_t(q[k]);
        c.tune.valu_nw[k] = uint8_t(nw[k]);
        c.tune.kara_base[k] = uint16_t(kb[k]);
        c.tune.list_algo[k] = la[k];
    }
    c.add.multi2 = m[0] != 0;
    c.add.multi4 = m[1] != 0;
    c.add.multi8 = m[2] != 0;
    return BI_OK;
}

}  // namespace bi
