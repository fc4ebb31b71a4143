// Context set-up and dispatch from the C ABI to the kernel launchers.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <algorithm>
#include <cstdlib>

#include "bi_internal.hpp"

namespace bi {

hipError_t lds_limit_once(const void *fn, std::atomic<uint64_t> &done) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const uint64_t bit = dev >= 0 && dev < 64 ? uint64_t(1) << dev : 0;
    if (bit && (done.load(std::memory_order_acquire) & bit)) return hipSuccess;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e == hipSuccess && bit) done.fetch_or(bit, std::memory_order_release);
    return e;
}

bool algo_supports(int algo, uint32_t n32) {
    switch (algo) {
        case BI_MUL_SCHOOL_VALU: return n32 >= 1 && n32 <= kMaxLimbs32;
        case BI_MUL_SCHOOL_MFMA: return n32 >= 1 && n32 <= kMaxLimbs32;
        case BI_MUL_NTT: return n32 >= 1 && ntt_log_len(n32) != 0;
        case BI_MUL_NTT_PF64: return n32 >= 1 && ntt64_log_len(n32) != 0;
        case BI_MUL_KARATSUBA: return n32 >= 1 && n32 <= kMaxLimbs32;
        default: return false;
    }
}

int resolve_algo(const Tune &tune, uint32_t n32, int algo) {
    if (algo != BI_MUL_AUTO) return algo;
    algo = tune.mul_algo[size_class_host(n32)];
    return algo_supports(algo, n32) ? algo : BI_MUL_SCHOOL_VALU;
}

int kara_base_algo(const Tune &tune, uint32_t h, bool ragged) {
    const uint32_t k = size_class_host(h);
    const int alg = ragged ? tune.list_algo[k] : tune.mul_algo[k];
    if (alg != BI_MUL_KARATSUBA && algo_supports(alg, h)) return alg;
    return BI_MUL_SCHOOL_MFMA;
}

size_t uniform_algo_scratch_bytes(int alg, uint32_t n32) {
    switch (alg) {
        case BI_MUL_SCHOOL_MFMA: return n32 <= mfma_max_limbs() ? 0 : mfma_big_slot_bytes(n32);
        case BI_MUL_NTT: return ntt_scratch_bytes(n32, 1);
        case BI_MUL_NTT_PF64: return ntt64_scratch_bytes(n32, 1);
        default: return 0;
    }
}

// Built-in per-class tables, as bi_autotune measured them on MI355X (one
// GPU, a fresh context).  Uniform batches, each class at its largest size:
// the VALU schoolbook up to 64 limbs (2^11 bits), the int8-MFMA schoolbook up
// to 4096 limbs (2^17 bits), the two-prime NTT at 8192 limbs.  Ragged batches
// (sizes spread over each class): the same up to 4096 limbs, Karatsuba over
// 8192 (its work follows each instance's size; an NTT's transform length is
// the class's).  Also the VALU schedule (Q output words per lane, waves per
// workgroup) per class.  bi_autotune re-measures and replaces them on the
// device at hand.
static void default_tune(Tune &t) {
    static const int algo[kNumClasses] = {BI_MUL_SCHOOL_VALU, BI_MUL_SCHOOL_VALU, BI_MUL_SCHOOL_VALU,
                                          BI_MUL_SCHOOL_MFMA, BI_MUL_SCHOOL_MFMA, BI_MUL_SCHOOL_MFMA,
                                          BI_MUL_SCHOOL_MFMA, BI_MUL_SCHOOL_MFMA, BI_MUL_SCHOOL_MFMA,
                                          BI_MUL_NTT};
    static const int list[kNumClasses] = {BI_MUL_SCHOOL_VALU, BI_MUL_SCHOOL_VALU, BI_MUL_SCHOOL_VALU,
                                          BI_MUL_SCHOOL_MFMA, BI_MUL_SCHOOL_MFMA, BI_MUL_SCHOOL_MFMA,
                                          BI_MUL_SCHOOL_MFMA, BI_MUL_SCHOOL_MFMA, BI_MUL_SCHOOL_MFMA,
                                          BI_MUL_KARATSUBA};
    static const uint8_t q[kNumClasses] = {2, 2, 2, 4, 2, 2, 4, 4, 4, 4};
    static const uint8_t nw[kNumClasses] = {1, 1, 1, 1, 2, 4, 4, 8, 16, 16};
    for (uint32_t k = 0; k < kNumClasses; ++k) {
        t.mul_algo[k] = algo[k];
        t.list_algo[k] = list[k];
        t.valu_q[k] = q[k];
        t.valu_nw[k] = nw[k];
        t.kara_base[k] = kKaraBase;
    }
}

KaraPlan kara_plan_tuned(const Tune &tune, uint32_t n32) {
    const uint32_t b = tune.kara_base[size_class_host(n32)];
    return kara_plan(n32, b ? b : kKaraBase);
}

bi_status ctx_init(Ctx &c, int device, const hipDeviceProp_t &prop) {
    c.device = device;
    std::snprintf(c.arch, sizeof(c.arch), "%s", prop.gcnArchName);
    if (hipRuntimeGetVersion(&c.hip_version) != hipSuccess) c.hip_version = 0;
    default_tune(c.tune);
    c.num_cus = prop.multiProcessorCount;
    // Defaults from a sweep on MI355X (u64 limbs, 1 GiB of operands): a large
    // grid, one wave per instance for 2-4 row instances, workgroup-cooperative
    // above (bi_autotune re-measures the row classes).
    c.add.max_waves = uint64_t(prop.multiProcessorCount) * 1024;
    c.add.multi2 = true;
    c.add.multi4 = true;
    c.add.multi8 = false;
    // Experiment override: BI_KARA_BASE=<words> sets every class's Karatsuba base.
    if (const char *env = std::getenv("BI_KARA_BASE")) {
        const int b = std::atoi(env);
        for (uint32_t v : kKaraBases)
            if (b == int(v))
                for (uint32_t k = 0; k < kNumClasses; ++k) c.tune.kara_base[k] = uint16_t(b);
    }
    // Experiment override: BI_ADD_TUNE="rows,nt,max_waves,multi_mask"
    // (e.g. "8,1,32768,7"; multi_mask bit 0/1/2 = 2/4/8-row instances).
    if (const char *env = std::getenv("BI_ADD_TUNE")) {
        int rows = 4, nt = 1, mm = 3;
        unsigned long long mw = c.add.max_waves;
        if (std::sscanf(env, "%d,%d,%llu,%d", &rows, &nt, &mw, &mm) >= 1) {
            c.add.rows = (rows == 2 || rows == 8) ? rows : 4;
            c.add.nt = nt != 0;
            c.add.max_waves = mw ? mw : c.add.max_waves;
            c.add.multi2 = mm & 1;
            c.add.multi4 = (mm >> 1) & 1;
            c.add.multi8 = (mm >> 2) & 1;
        }
    }
    return ntt_setup(c.ntt);
}

void ctx_release(Ctx &c) {
    ntt_release(c.ntt);
    if (c.scratch.ptr) (void)hipFree(c.scratch.ptr);
    c.scratch = Scratch{};
}

bi_status ctx_scratch(Ctx &c, size_t bytes, hipStream_t st, void **out) {
    if (bytes <= c.scratch.bytes) {
        *out = c.scratch.ptr;
        return BI_OK;
    }
    if (c.scratch.ptr) {
        // Every stream that used the old buffer must be done with it, not
        // only `st`: growth is rare, so wait for the whole device.
        (void)st;
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return set_error(BI_EHIP, "scratch resize: %s", hipGetErrorString(e));
        (void)hipFree(c.scratch.ptr);
        c.scratch = Scratch{};
    }
    const size_t want = bytes + bytes / 4;  // headroom against repeated growth
    void *p = nullptr;
    if (hipMalloc(&p, want) != hipSuccess) return set_error(BI_ENOMEM, "scratch allocation of %zu bytes failed", want);
    c.scratch.ptr = p;
    c.scratch.bytes = want;
    *out = p;
    return BI_OK;
}

bi_status dispatch_bigadd_v(Ctx &c, const void *a, const void *b, void *out, uint8_t *carry, const bi_desc *desc,
                            uint64_t count, uint32_t limb_bits, hipStream_t st) {
    hipError_t e = launch_bigadd_ragged(a, b, out, carry, desc, count, limb_bits, st, c.add);
    if (e != hipSuccess) return set_error(BI_EHIP, "bigadd_v launch: %s", hipGetErrorString(e));
    return BI_OK;
}

uint32_t size_class_host(uint32_t n32) {
    uint32_t k = 0;
    while (k + 1 < kNumClasses && class_nmax(k) < n32) ++k;
    return k;
}

// Scratch for `per_inst` bytes per product of a batch: the fixed buffer when
// given (rounds of as many products as it holds), else the context's buffer
// grown to the whole batch.
static bi_status bigmul_scratch(Ctx &c, size_t per_inst, uint64_t batch, hipStream_t st, void *fixed,
                                size_t fixed_bytes, void **scr, uint64_t *round) {
    if (fixed) {
        if (per_inst > fixed_bytes)
            return set_error(BI_ESIZE, "one product needs %zu bytes of scratch, the fixed array holds %zu", per_inst,
                             fixed_bytes);
        *scr = fixed;
        *round = fixed_bytes / per_inst;
        return BI_OK;
    }
    *round = batch;
    return ctx_scratch(c, per_inst * size_t(batch), st, scr);
}

bi_status dispatch_bigmul(Ctx &c, const void *a, const void *b, void *out, uint32_t n32, uint64_t batch, int algo,
                          hipStream_t st, void *fixed, size_t fixed_bytes) {
    algo = resolve_algo(c.tune, n32, algo);
    auto A = static_cast<const uint32_t *>(a);
    auto B = static_cast<const uint32_t *>(b);
    auto C = static_cast<uint32_t *>(out);
    hipError_t e = hipSuccess;
    void *scr = nullptr;
    uint64_t round = 0;
    bi_status s = BI_OK;
    switch (algo) {
        case BI_MUL_SCHOOL_VALU:
            e = launch_bigmul_valu(A, B, C, n32, batch, valu_plan_tuned(n32, c.tune), st, c.num_cus);
            break;
        case BI_MUL_SCHOOL_MFMA:
            if (n32 <= mfma_max_limbs()) {
                e = launch_bigmul_mfma(A, B, C, n32, batch, st, c.num_cus);
            } else {
                s = bigmul_scratch(c, mfma_big_slot_bytes(n32), batch, st, fixed, fixed_bytes, &scr, &round);
                if (s != BI_OK) return s;
                e = launch_bigmul_mfma_big(A, B, C, n32, batch, static_cast<uint8_t *>(scr), st, c.num_cus, round);
            }
            break;
        case BI_MUL_NTT:
            if (ntt_log_len(n32) == 0) return set_error(BI_EALGO, "NTT supports up to %u limbs", kNttLmax / 4);
            s = bigmul_scratch(c, ntt_scratch_bytes(n32, 1), batch, st, fixed, fixed_bytes, &scr, &round);
            if (s != BI_OK) return s;
            e = launch_bigmul_ntt(c.ntt.c, A, B, C, n32, batch, static_cast<uint32_t *>(scr), st, round, c.num_cus);
            break;
        case BI_MUL_NTT_PF64:
            if (ntt64_log_len(n32) == 0)
                return set_error(BI_EALGO, "NTT (PrimeField64) supports up to %u limbs", kP64Hmax / 2);
            s = bigmul_scratch(c, ntt64_scratch_bytes(n32, 1), batch, st, fixed, fixed_bytes, &scr, &round);
            if (s != BI_OK) return s;
            e = launch_bigmul_ntt64(c.ntt.c64, A, B, C, n32, batch, static_cast<uint64_t *>(scr), st, round);
            break;
        case BI_MUL_KARATSUBA: {
            const KaraPlan kp = kara_plan_tuned(c.tune, n32);
            const uint32_t hb = kp.h[kp.levels];
            const int base = kara_base_algo(c.tune, hb);
            uint64_t nbase = 1;  // base products per instance
            for (int j = 0; j < kp.levels; ++j) nbase *= 3;
            // the base's own scratch: all of a round's products at once
            const size_t per_base = uniform_algo_scratch_bytes(base, hb);
            const size_t per = kara_round_bytes(kp, 1, false, per_base * nbase);
            uint64_t R = batch;
            if (fixed) {
                R = std::min<uint64_t>(batch, fixed_bytes / per);
                if (R == 0)
                    return set_error(BI_ESIZE, "one Karatsuba product needs %zu bytes of scratch, the fixed array "
                                     "holds %zu", per, fixed_bytes);
                while (R > 1 && kara_round_bytes(kp, R, false, per_base * nbase * R) > fixed_bytes) --R;
                scr = fixed;
            } else {
                // rounds of at most kKaraScratchBudget bytes (at least one instance)
                R = std::min<uint64_t>(batch, std::max<uint64_t>(1, kKaraScratchBudget / per));
                s = ctx_scratch(c, kara_round_bytes(kp, R, false, per_base * nbase * R), st, &scr);
                if (s != BI_OK) return s;
            }
            return launch_bigmul_kara(c, A, B, C, n32, batch, kp, base, per_base * nbase * R,
                                      static_cast<uint8_t *>(scr), R, st);
        }
        default:
            return set_error(BI_EALGO, "multiplication algorithm %d is not available", algo);
    }
    if (e != hipSuccess) return set_error(BI_EHIP, "bigmul launch: %s", hipGetErrorString(e));
    return BI_OK;
}

}  // namespace bi
