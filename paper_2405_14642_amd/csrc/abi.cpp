// C ABI of the library: argument validation (host only, before any HIP call)
// and dispatch to the kernel launchers.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "bi_internal.hpp"

namespace {
thread_local char g_err[512] = "";
}

namespace bi {
bi_status set_error(bi_status s, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return s;
}
}  // namespace bi

namespace {

template <typename... Args>
bi_status fail(bi_status s, const char *fmt, Args... args) {
    return bi::set_error(s, fmt, args...);
}

bi_status hip_fail(hipError_t e, const char *what) {
    return fail(BI_EHIP, "%s: %s", what, hipGetErrorString(e));
}

bool overlaps(const void *p, uint64_t pn, const void *q, uint64_t qn) {
    if (!p || !q || pn == 0 || qn == 0) return false;
    const uintptr_t a = reinterpret_cast<uintptr_t>(p), b = reinterpret_cast<uintptr_t>(q);
    return a < b + qn && b < a + pn;
}

// Common shape checks for uniform batches.  On success *bytes = bytes per operand.
bi_status check_shape(uint32_t n_limbs, uint32_t limb_bits, uint64_t batch, uint64_t *inst_bytes) {
    if (limb_bits != 32 && limb_bits != 64) return fail(BI_ELIMB, "limb_bits must be 32 or 64 (got %u)", limb_bits);
    if (n_limbs == 0) return fail(BI_EINVAL, "n_limbs must be >= 1");
    if (uint64_t(n_limbs) * limb_bits > BI_MAX_BITS)
        return fail(BI_ESIZE, "n_limbs * limb_bits = %llu exceeds %u bits",
                    (unsigned long long)(uint64_t(n_limbs) * limb_bits), BI_MAX_BITS);
    *inst_bytes = uint64_t(n_limbs) * (limb_bits / 8);
    if (batch > (uint64_t(1) << 40) / *inst_bytes) return fail(BI_ESIZE, "batch too large");
    return BI_OK;
}

bi_status check_ptr(const void *p, uint32_t limb_bits, const char *name) {
    if (!p) return fail(BI_EINVAL, "%s is NULL", name);
    if (reinterpret_cast<uintptr_t>(p) % (limb_bits / 8))
        return fail(BI_ELIMB, "%s is not aligned to %u-bit limbs", name, limb_bits);
    return BI_OK;
}

using bi::DeviceGuard;

}  // namespace

extern "C" {

const char *bi_status_str(int s) {
    switch (s) {
        case BI_OK: return "ok";
        case BI_EINVAL: return "invalid argument";
        case BI_ESIZE: return "size out of range";
        case BI_ELIMB: return "bad limb width or alignment";
        case BI_EALIAS: return "output overlaps an input";
        case BI_EHIP: return "HIP runtime error";
        case BI_ENOMEM: return "device allocation failed";
        case BI_EALGO: return "algorithm unavailable for this size";
        case BI_ENODEV: return "no usable gfx950 device";
        default: return "unknown status";
    }
}

const char *bi_last_error(void) { return g_err; }

bi_status bi_ctx_create(int device, bi_ctx **out) {
    if (!out) return fail(BI_EINVAL, "out is NULL");
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return fail(BI_ENODEV, "no HIP device");
    if (device < 0 || device >= count) return fail(BI_ENODEV, "device %d out of range (%d devices)", device, count);
    hipDeviceProp_t prop;
    hipError_t e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(BI_ENODEV, "device %d is %s, not gfx950", device, prop.gcnArchName);
    bi_ctx *c = new (std::nothrow) bi_ctx;
    if (!c) return fail(BI_ENOMEM, "host allocation failed");
    c->device = device;
    DeviceGuard g(device);
    if (g.err != hipSuccess) {
        delete c;
        return hip_fail(g.err, "hipSetDevice");
    }
    bi_status st = bi::ctx_init(c->impl, device, prop);
    if (st == BI_OK) st = bi::fixed_scratch_init(device, &c->impl.fixed_scratch);
    if (st != BI_OK) {
        bi::ctx_release(c->impl);
        delete c;
        return st == BI_ENOMEM ? fail(st, "device table allocation failed") : fail(st, "context set-up failed");
    }
    *out = c;
    return BI_OK;
}

void bi_ctx_destroy(bi_ctx *ctx) {
    if (!ctx) return;
    {
        DeviceGuard g(ctx->device);
        bi::ctx_release(ctx->impl);
    }
    delete ctx;
}

bi_status bigadd(bi_ctx *ctx, const void *a, const void *b, void *out, uint8_t *carry_out, uint32_t n_limbs,
                 uint32_t limb_bits, uint64_t batch, void *stream) {
    uint64_t ib = 0;
    bi_status s = check_shape(n_limbs, limb_bits, batch, &ib);
    if (s != BI_OK) return s;
    if (batch == 0) return ctx ? BI_OK : fail(BI_EINVAL, "ctx is NULL");
    if ((s = check_ptr(a, limb_bits, "a")) != BI_OK) return s;
    if ((s = check_ptr(b, limb_bits, "b")) != BI_OK) return s;
    if ((s = check_ptr(out, limb_bits, "out")) != BI_OK) return s;
    const uint64_t tot = ib * batch;
    if (out != a && overlaps(out, tot, a, tot)) return fail(BI_EALIAS, "out partially overlaps a");
    if (out != b && overlaps(out, tot, b, tot)) return fail(BI_EALIAS, "out partially overlaps b");
    if (overlaps(carry_out, batch, a, tot) || overlaps(carry_out, batch, b, tot) || overlaps(carry_out, batch, out, tot))
        return fail(BI_EALIAS, "carry_out overlaps an operand");
    if (!ctx) return fail(BI_EINVAL, "ctx is NULL");
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    hipError_t e = bi::launch_bigadd(a, b, out, carry_out, ib, batch, static_cast<hipStream_t>(stream), ctx->impl.add);
    if (e != hipSuccess) return hip_fail(e, "bigadd launch");
    return BI_OK;
}

bi_status bigadd_large(bi_ctx *ctx, const void *a, const void *b, void *out, uint8_t *carry_out, uint64_t n_limbs,
                       uint32_t limb_bits, void *stream) {
    if (limb_bits != 32 && limb_bits != 64) return fail(BI_ELIMB, "limb_bits must be 32 or 64 (got %u)", limb_bits);
    if (n_limbs == 0) return fail(BI_EINVAL, "n_limbs must be >= 1");
    if (n_limbs > BI_MAX_LARGE_BITS / limb_bits)
        return fail(BI_ESIZE, "n_limbs * limb_bits exceeds 2^40 bits (n_limbs = %llu)", (unsigned long long)n_limbs);
    bi_status s;
    if ((s = check_ptr(a, limb_bits, "a")) != BI_OK) return s;
    if ((s = check_ptr(b, limb_bits, "b")) != BI_OK) return s;
    if ((s = check_ptr(out, limb_bits, "out")) != BI_OK) return s;
    const uint64_t tot = n_limbs * (limb_bits / 8);
    if (out != a && overlaps(out, tot, a, tot)) return fail(BI_EALIAS, "out partially overlaps a");
    if (out != b && overlaps(out, tot, b, tot)) return fail(BI_EALIAS, "out partially overlaps b");
    if (overlaps(carry_out, 1, a, tot) || overlaps(carry_out, 1, b, tot) || overlaps(carry_out, 1, out, tot))
        return fail(BI_EALIAS, "carry_out overlaps an operand");
    if (!ctx) return fail(BI_EINVAL, "ctx is NULL");
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const uint64_t n32 = n_limbs * (limb_bits / 32);
    const uint64_t tiles = bi::large_add_tiles(n32, bi::large_add_chunk_words(a, b, out));
    void *scr = nullptr;
    if ((s = bi::ctx_scratch(ctx->impl, bi::large_add_scratch_bytes(tiles), st, &scr)) != BI_OK) return s;
    hipError_t e = bi::launch_bigadd_large(a, b, out, carry_out, n32, static_cast<uint8_t *>(scr), st,
                                           ctx->impl.num_cus);
    if (e != hipSuccess) return hip_fail(e, "bigadd_large launch");
    return BI_OK;
}

bi_status bi_mul_large_plan(uint64_t n_limbs, uint32_t limb_bits, int algo, uint32_t *block_bits, uint32_t *blocks) {
    if (limb_bits != 32 && limb_bits != 64) return fail(BI_ELIMB, "limb_bits must be 32 or 64 (got %u)", limb_bits);
    if (n_limbs == 0) return fail(BI_EINVAL, "n_limbs must be >= 1");
    if (n_limbs > BI_MAX_LARGE_MUL_BITS / limb_bits)
        return fail(BI_ESIZE, "n_limbs * limb_bits exceeds %u bits (n_limbs = %llu)", BI_MAX_LARGE_MUL_BITS,
                    (unsigned long long)n_limbs);
    if (algo < BI_MUL_AUTO || algo > BI_MUL_KARATSUBA) return fail(BI_EINVAL, "unknown algorithm %d", algo);
    if (!block_bits || !blocks) return fail(BI_EINVAL, "NULL argument");
    const uint64_t n32 = n_limbs * (limb_bits / 32);
    const bool two_dim = algo == BI_MUL_AUTO || algo == BI_MUL_NTT;
    const uint32_t bw = two_dim ? bi::large_ntt_auto_block(n32) : bi::large_mul_auto_block(n32);
    *block_bits = 32 * bw;
    *blocks = uint32_t((n32 + bw - 1) / bw);
    return BI_OK;
}

bi_status bigmul_large(bi_ctx *ctx, const void *a, const void *b, void *out, uint64_t n_limbs, uint32_t limb_bits,
                       int algo, uint32_t block_bits, void *stream) {
    if (limb_bits != 32 && limb_bits != 64) return fail(BI_ELIMB, "limb_bits must be 32 or 64 (got %u)", limb_bits);
    if (n_limbs == 0) return fail(BI_EINVAL, "n_limbs must be >= 1");
    if (n_limbs > BI_MAX_LARGE_MUL_BITS / limb_bits)
        return fail(BI_ESIZE, "n_limbs * limb_bits exceeds %u bits (n_limbs = %llu)", BI_MAX_LARGE_MUL_BITS,
                    (unsigned long long)n_limbs);
    if (algo < BI_MUL_AUTO || algo > BI_MUL_KARATSUBA) return fail(BI_EINVAL, "unknown algorithm %d", algo);
    const uint64_t n32 = n_limbs * (limb_bits / 32);
    // AUTO and NTT: the two-dimensional NTT convolution (n log n); a forced
    // VALU, MFMA or PrimeField64 algorithm: k^2 block products of that algorithm.
    const bool two_dim = algo == BI_MUL_AUTO || algo == BI_MUL_NTT;
    uint32_t bw = 0;
    if (two_dim) {
        if (block_bits != 0 && (block_bits < (1u << 14) || block_bits > (1u << 18) || (block_bits & (block_bits - 1))))
            return fail(BI_EINVAL, "block_bits must be 0 or a power of two in [2^14, 2^18] (got %u)", block_bits);
        bw = block_bits ? block_bits / 32 : bi::large_ntt_auto_block(n32);
        if ((n32 + bw - 1) / bw > bi::kLargeNttMaxBlocks)
            return fail(BI_EINVAL, "%u-bit blocks give more than %u blocks at %llu words", 32 * bw,
                        bi::kLargeNttMaxBlocks, (unsigned long long)n32);
    } else {
        if (block_bits != 0 && block_bits != (1u << 16) && block_bits != (1u << 17) && block_bits != (1u << 18))
            return fail(BI_EINVAL, "block_bits must be 0, 2^16, 2^17 or 2^18 for block products (got %u)", block_bits);
        bw = block_bits ? block_bits / 32 : bi::large_mul_auto_block(n32);
        if (!bi::algo_supports(algo, bw)) return fail(BI_EALGO, "algorithm %d does not run %u-bit blocks", algo, 32 * bw);
    }
    bi_status s;
    if ((s = check_ptr(a, limb_bits, "a")) != BI_OK) return s;
    if ((s = check_ptr(b, limb_bits, "b")) != BI_OK) return s;
    if ((s = check_ptr(out, limb_bits, "out")) != BI_OK) return s;
    const uint64_t tot = n_limbs * (limb_bits / 8);
    if (overlaps(out, 2 * tot, a, tot) || overlaps(out, 2 * tot, b, tot)) return fail(BI_EALIAS, "out overlaps an input");
    if (!ctx) return fail(BI_EINVAL, "ctx is NULL");
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    const hipStream_t st = static_cast<hipStream_t>(stream);
    void *scr = nullptr;
    const size_t need =
        two_dim ? bi::large_ntt_scratch_bytes(n32, bw) : bi::large_mul_scratch_bytes(n32, bw, ctx->impl.num_cus);
    if ((s = bi::ctx_scratch(ctx->impl, need, st, &scr)) != BI_OK) return s;
    auto A = static_cast<const uint32_t *>(a);
    auto B = static_cast<const uint32_t *>(b);
    auto C = static_cast<uint32_t *>(out);
    auto S = static_cast<uint8_t *>(scr);
    const hipError_t e = two_dim ? bi::launch_bigmul_large_ntt(ctx->impl, A, B, C, n32, bw, S, st)
                                 : bi::launch_bigmul_large(ctx->impl, A, B, C, n32, bw, algo, S, st);
    if (e != hipSuccess) return hip_fail(e, "bigmul_large launch");
    return BI_OK;
}

// bigmul's argument checks; *n32 receives the operands' 32-bit words.
static bi_status check_bigmul(bi_ctx *ctx, const void *a, const void *b, const void *out, uint32_t n_limbs,
                              uint32_t limb_bits, uint64_t batch, int algo, uint32_t *n32) {
    uint64_t ib = 0;
    bi_status s = check_shape(n_limbs, limb_bits, batch, &ib);
    if (s != BI_OK) return s;
    if (algo < BI_MUL_AUTO || algo > BI_MUL_KARATSUBA) return fail(BI_EINVAL, "unknown algorithm %d", algo);
    if (batch > 0) {
        if ((s = check_ptr(a, limb_bits, "a")) != BI_OK) return s;
        if ((s = check_ptr(b, limb_bits, "b")) != BI_OK) return s;
        if ((s = check_ptr(out, limb_bits, "out")) != BI_OK) return s;
        const uint64_t tot = ib * batch;
        if (overlaps(out, 2 * tot, a, tot) || overlaps(out, 2 * tot, b, tot))
            return fail(BI_EALIAS, "out overlaps an input");
    }
    if (!ctx) return fail(BI_EINVAL, "ctx is NULL");
    // The multiplication kernels work on 32-bit limbs; 64-bit limbs are the
    // same byte string with twice as many limbs.
    *n32 = n_limbs * (limb_bits / 32);
    return BI_OK;
}

bi_status bigmul(bi_ctx *ctx, const void *a, const void *b, void *out, uint32_t n_limbs, uint32_t limb_bits,
                 uint64_t batch, int algo, void *stream) {
    uint32_t n32 = 0;
    const bi_status s = check_bigmul(ctx, a, b, out, n_limbs, limb_bits, batch, algo, &n32);
    if (s != BI_OK || batch == 0) return s;
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    return bi::dispatch_bigmul(ctx->impl, a, b, out, n32, batch, algo, static_cast<hipStream_t>(stream));
}

bi_status bigmul_noalloc(bi_ctx *ctx, const void *a, const void *b, void *out, uint32_t n_limbs, uint32_t limb_bits,
                         uint64_t batch, int algo, void *stream) {
    uint32_t n32 = 0;
    const bi_status s = check_bigmul(ctx, a, b, out, n_limbs, limb_bits, batch, algo, &n32);
    if (s != BI_OK || batch == 0) return s;
    if (!ctx->impl.fixed_scratch) return fail(BI_EHIP, "the context has no fixed scratch array");
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    // every scratch buffer from the fixed array (batches run in rounds that
    // fit it; BI_ESIZE if one product does not)
    return bi::dispatch_bigmul(ctx->impl, a, b, out, n32, batch, algo, static_cast<hipStream_t>(stream),
                               ctx->impl.fixed_scratch, bi::kFixedScratchBytes);
}

bi_status bi_fused(bi_ctx *ctx, int program, const void *a, const void *b, void *out, uint32_t n_limbs,
                   uint32_t limb_bits, uint64_t batch, void *stream) {
    uint64_t ib = 0;
    bi_status s = check_shape(n_limbs, limb_bits, batch, &ib);
    if (s != BI_OK) return s;
    if (program < BI_PROG_ADD6 || program > BI_PROG_MUL_LOW) return fail(BI_EINVAL, "unknown program %d", program);
    if (batch == 0) return ctx ? BI_OK : fail(BI_EINVAL, "ctx is NULL");
    if ((s = check_ptr(a, limb_bits, "a")) != BI_OK) return s;
    if ((s = check_ptr(b, limb_bits, "b")) != BI_OK) return s;
    if ((s = check_ptr(out, limb_bits, "out")) != BI_OK) return s;
    const uint64_t tot = ib * batch;
    if (overlaps(out, tot, a, tot) || overlaps(out, tot, b, tot)) return fail(BI_EALIAS, "out overlaps an input");
    if (!ctx) return fail(BI_EINVAL, "ctx is NULL");
    const uint32_t n32 = n_limbs * (limb_bits / 32);
    if (bi::fused_lds_bytes(program, n32) > 160 * 1024)
        return fail(BI_ESIZE, "program %d does not fit one workgroup's LDS at %u words", program, n32);
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    const hipError_t e = bi::launch_fused(program, static_cast<const uint32_t *>(a), static_cast<const uint32_t *>(b),
                                          static_cast<uint32_t *>(out), n32, batch, static_cast<hipStream_t>(stream),
                                          ctx->impl.num_cus);
    if (e != hipSuccess) return hip_fail(e, "fused program launch");
    return BI_OK;
}

bi_status bigadd_v(bi_ctx *ctx, const void *a, const void *b, void *out, uint8_t *carry_out, const bi_desc *desc,
                   uint64_t count, uint32_t limb_bits, void *stream) {
    if (limb_bits != 32 && limb_bits != 64) return fail(BI_ELIMB, "limb_bits must be 32 or 64 (got %u)", limb_bits);
    if (count == 0) return ctx ? BI_OK : fail(BI_EINVAL, "ctx is NULL");
    if (!desc) return fail(BI_EINVAL, "desc is NULL");
    bi_status s;
    if ((s = check_ptr(a, limb_bits, "a")) != BI_OK) return s;
    if ((s = check_ptr(b, limb_bits, "b")) != BI_OK) return s;
    if ((s = check_ptr(out, limb_bits, "out")) != BI_OK) return s;
    if (reinterpret_cast<uintptr_t>(desc) % alignof(bi_desc)) return fail(BI_EINVAL, "desc is not 8-byte aligned");
    if (!ctx) return fail(BI_EINVAL, "ctx is NULL");
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    return bi::dispatch_bigadd_v(ctx->impl, a, b, out, carry_out, desc, count, limb_bits, static_cast<hipStream_t>(stream));
}

bi_status bigmul_v(bi_ctx *ctx, const void *a, const void *b, void *out, const bi_desc *desc, uint64_t count,
                   uint32_t limb_bits, int algo, void *stream) {
    if (limb_bits != 32 && limb_bits != 64) return fail(BI_ELIMB, "limb_bits must be 32 or 64 (got %u)", limb_bits);
    if (algo < BI_MUL_AUTO || algo > BI_MUL_KARATSUBA) return fail(BI_EINVAL, "unknown algorithm %d", algo);
    if (count == 0) return ctx ? BI_OK : fail(BI_EINVAL, "ctx is NULL");
    if (!desc) return fail(BI_EINVAL, "desc is NULL");
    bi_status s;
    if ((s = check_ptr(a, limb_bits, "a")) != BI_OK) return s;
    if ((s = check_ptr(b, limb_bits, "b")) != BI_OK) return s;
    if ((s = check_ptr(out, limb_bits, "out")) != BI_OK) return s;
    if (reinterpret_cast<uintptr_t>(desc) % alignof(bi_desc)) return fail(BI_EINVAL, "desc is not 8-byte aligned");
    if (!ctx) return fail(BI_EINVAL, "ctx is NULL");
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    return bi::dispatch_bigmul_v(ctx->impl, a, b, out, desc, count, limb_bits, algo, static_cast<hipStream_t>(stream));
}

bi_status bi_autotune(bi_ctx *ctx, void *stream, int *algo_out, uint32_t n_out) {
    if (!ctx) return fail(BI_EINVAL, "ctx is NULL");
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    return bi::autotune(ctx->impl, static_cast<hipStream_t>(stream), algo_out, n_out);
}

bi_status bi_tune_get(const bi_ctx *ctx, int *algo_out, uint32_t n_out) {
    if (!ctx || !algo_out) return fail(BI_EINVAL, "NULL argument");
    for (uint32_t k = 0; k < n_out && k < bi::kNumClasses; ++k) algo_out[k] = ctx->impl.tune.mul_algo[k];
    return BI_OK;
}

bi_status bi_mul_plan(const bi_ctx *ctx, uint32_t n_limbs, uint32_t limb_bits, int algo, bi_mul_plan_info *out) {
    uint64_t ib = 0;
    bi_status s = check_shape(n_limbs, limb_bits, 1, &ib);
    if (s != BI_OK) return s;
    if (algo < BI_MUL_AUTO || algo > BI_MUL_KARATSUBA) return fail(BI_EINVAL, "unknown algorithm %d", algo);
    if (!ctx || !out) return fail(BI_EINVAL, "NULL argument");
    const uint32_t n32 = n_limbs * (limb_bits / 32);
    const int alg = bi::resolve_algo(ctx->impl.tune, n32, algo);
    if (!bi::algo_supports(alg, n32)) return fail(BI_EALGO, "algorithm %d does not run %u-word products", alg, n32);
    bi_mul_plan_info r{};
    r.algo = alg;
    r.base_limbs = n32;
    r.base_algo = alg;
    if (alg == BI_MUL_KARATSUBA) {
        const bi::KaraPlan kp = bi::kara_plan_tuned(ctx->impl.tune, n32);
        r.kara_levels = kp.levels;
        r.base_limbs = kp.h[kp.levels];
        r.base_algo = bi::kara_base_algo(ctx->impl.tune, r.base_limbs);
    }
    *out = r;
    return BI_OK;
}

bi_status bi_tune_get_list(const bi_ctx *ctx, int *algo_out, uint32_t n_out) {
    if (!ctx || !algo_out) return fail(BI_EINVAL, "NULL argument");
    for (uint32_t k = 0; k < n_out && k < bi::kNumClasses; ++k) algo_out[k] = ctx->impl.tune.list_algo[k];
    return BI_OK;
}

bi_status bi_tune_set_list(bi_ctx *ctx, const int *algo_in, uint32_t n_in) {
    if (!ctx || !algo_in) return fail(BI_EINVAL, "NULL argument");
    for (uint32_t k = 0; k < n_in && k < bi::kNumClasses; ++k)
        if (!bi::algo_supports(algo_in[k], bi::class_nmax(k)))
            return fail(BI_EALGO, "algorithm %d cannot run size class %u", algo_in[k], k);
    for (uint32_t k = 0; k < n_in && k < bi::kNumClasses; ++k) ctx->impl.tune.list_algo[k] = algo_in[k];
    return BI_OK;
}

bi_status bi_tune_get_kara(const bi_ctx *ctx, uint32_t *base_out, uint32_t n_out) {
    if (!ctx || !base_out) return fail(BI_EINVAL, "NULL argument");
    for (uint32_t k = 0; k < n_out && k < bi::kNumClasses; ++k) base_out[k] = ctx->impl.tune.kara_base[k];
    return BI_OK;
}

bi_status bi_tune_set_kara(bi_ctx *ctx, const uint32_t *base_in, uint32_t n_in) {
    if (!ctx || !base_in) return fail(BI_EINVAL, "NULL argument");
    for (uint32_t k = 0; k < n_in && k < bi::kNumClasses; ++k)
        if (!bi::kara_base_valid(base_in[k]))
            return fail(BI_EINVAL, "Karatsuba base %u of class %u is not 512, 1024 or 2048", base_in[k], k);
    for (uint32_t k = 0; k < n_in && k < bi::kNumClasses; ++k) ctx->impl.tune.kara_base[k] = uint16_t(base_in[k]);
    return BI_OK;
}

bi_status bi_tune_save(const bi_ctx *ctx, const char *path) {
    if (!ctx || !path) return fail(BI_EINVAL, "NULL argument");
    return bi::tune_save(ctx->impl, path);
}

bi_status bi_tune_load(bi_ctx *ctx, const char *path) {
    if (!ctx || !path) return fail(BI_EINVAL, "NULL argument");
    return bi::tune_load(ctx->impl, path);
}

bi_status bi_tune_set(bi_ctx *ctx, const int *algo_in, uint32_t n_in) {
    if (!ctx || !algo_in) return fail(BI_EINVAL, "NULL argument");
    for (uint32_t k = 0; k < n_in && k < bi::kNumClasses; ++k)
        if (!bi::algo_supports(algo_in[k], bi::class_nmax(k)))
            return fail(BI_EALGO, "algorithm %d cannot run size class %u", algo_in[k], k);
    for (uint32_t k = 0; k < n_in && k < bi::kNumClasses; ++k) ctx->impl.tune.mul_algo[k] = algo_in[k];
    return BI_OK;
}

bi_status bi_tune_set_valu(bi_ctx *ctx, const int *q_in, const int *waves_in, uint32_t n_in) {
    if (!ctx || !q_in || !waves_in) return fail(BI_EINVAL, "NULL argument");
    const uint32_t m = n_in < bi::kNumClasses ? n_in : bi::kNumClasses;
    for (uint32_t k = 0; k < m; ++k) {
        if (q_in[k] == 0 && waves_in[k] == 0) continue;
        if (!bi::valu_plan_fits(bi::class_nmax(k), q_in[k], waves_in[k], nullptr))
            return fail(BI_EINVAL, "class %u: schedule (Q %d, %d waves) is not valid for its sizes", k, q_in[k],
                        waves_in[k]);
    }
    for (uint32_t k = 0; k < m; ++k) {
        ctx->impl.tune.valu_q[k] = uint8_t(q_in[k]);
        ctx->impl.tune.valu_nw[k] = uint8_t(waves_in[k]);
    }
    return BI_OK;
}

bi_status bi_tune_get_valu(const bi_ctx *ctx, int *q_out, int *waves_out, uint32_t n_out) {
    if (!ctx) return fail(BI_EINVAL, "ctx is NULL");
    for (uint32_t k = 0; k < n_out && k < bi::kNumClasses; ++k) {
        if (q_out) q_out[k] = ctx->impl.tune.valu_q[k];
        if (waves_out) waves_out[k] = ctx->impl.tune.valu_nw[k];
    }
    return BI_OK;
}

}  // extern "C"
