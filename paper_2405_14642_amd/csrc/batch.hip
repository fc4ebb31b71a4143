// Ragged multiplication batches (bigmul_v): device-side binning of the
// descriptors into size classes, then one launch per class of the kernel the
// class's algorithm names, each reading its instances from the class list.
// Everything is stream-ordered (no host synchronisation), so a whole ragged
// batch can be captured into a HIP graph and replayed.
#include <algorithm>

#include "bi_common.hpp"
#include "bi_internal.hpp"

namespace bi {

// Class c holds instances of (16 << (c-1), 16 << c] 32-bit limbs (class 0: <= 16).
__host__ __device__ inline uint32_t size_class(uint32_t n32) {
    if (n32 <= 16) return 0;
    return 32 - __builtin_clz(n32 - 1) - 4;
}
uint32_t class_nmax(uint32_t c) { return 16u << c; }

__global__ void zero_words_kernel(uint32_t *p, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

// counts[c] (pre-zeroed) and lists[c * stride + slot]: descriptor indices of
// class c.  The descriptor count is `count`, or *count_ptr when count_ptr is
// set (read on the device, clamped to `stride`).  Descriptors with 0 limbs or
// more than 8192 32-bit limbs are skipped.
__global__ void bin_kernel(const bi_desc *__restrict__ desc, uint64_t count, const uint64_t *count_ptr,
                           uint32_t words_per_limb, uint32_t *counts, uint32_t *lists, uint64_t stride) {
    if (count_ptr) count = min(*count_ptr, stride);
    const uint32_t lane = lane_id();
    const uint64_t below = (uint64_t(1) << lane) - 1;  // lanes under this one
    const uint64_t step = uint64_t(gridDim.x) * blockDim.x;
    // whole wavefronts walk the descriptors together, so the ballots below
    // see every lane of the wave
    for (uint64_t i0 = uint64_t(blockIdx.x) * blockDim.x + (threadIdx.x & ~63u); i0 < count; i0 += step) {
        const uint64_t i = i0 + lane;
        uint32_t c = kNumClasses;  // no class: past the end, or a skipped descriptor
        if (i < count) {
            const uint32_t n32 = desc[i].n_limbs * words_per_limb;
            if (n32 != 0 && n32 <= kMaxLimbs32) c = size_class(n32);
        }
        // one atomic per class present in the wave: the lowest lane of the
        // class reserves the slots, each lane takes its rank among them
        uint64_t todo = __ballot(c < kNumClasses);
        while (todo) {
            const uint32_t leader = uint32_t(__ffsll(static_cast<unsigned long long>(todo)) - 1);
            const uint32_t cl = __shfl(c, int(leader));
            const uint64_t same = __ballot(c == cl);
            uint32_t base = 0;
            if (lane == leader) base = atomicAdd(&counts[cl], uint32_t(__popcll(same)));
            base = __shfl(base, int(leader));
            if (c == cl) lists[uint64_t(cl) * stride + base + uint32_t(__popcll(same & below))] = uint32_t(i);
            todo &= ~same;
        }
    }
}

// counts (256 B), class lists, then the NTT transforms (256-byte aligned).
static size_t lists_bytes(uint64_t count) {
    return (size_t(kNumClasses) * count * sizeof(uint32_t) + 255) & ~size_t(255);
}

// Scratch a class launch may use for `count` instances: the largest of the
// NTT transforms and the Karatsuba levels (whatever the class's algorithm).
static size_t class_scratch_bytes(uint64_t count) {
    return std::max({ntt_list_scratch_bytes(count), ntt64_list_scratch_bytes(count), kara_list_scratch_bound(count)});
}

size_t batch_scratch_bytes(uint64_t count, int num_cus) {
    (void)num_cus;
    return 256 + lists_bytes(count) + class_scratch_bytes(count);
}

size_t list_algo_scratch_bytes(int alg, uint32_t nmax, uint64_t count) {
    switch (alg) {
        case BI_MUL_SCHOOL_MFMA: return nmax <= mfma_max_limbs() ? 0 : ntt_list_scratch_bytes(count);
        case BI_MUL_NTT: return ntt_list_scratch_bytes(count);
        case BI_MUL_NTT_PF64: return ntt64_list_scratch_bytes(count);
        default: return 0;
    }
}

hipError_t launch_bigmul_list_algo(const Ctx &c, const Tune &tune, const ListInst &src, uint32_t nmax,
                                   uint64_t count_max, int alg, void *scr, size_t scr_bytes, hipStream_t st) {
    switch (alg) {
        case BI_MUL_SCHOOL_MFMA:
            return nmax <= mfma_max_limbs() ? launch_bigmul_mfma_list(src, nmax, count_max, st, c.num_cus)
                                            : launch_bigmul_mfma_big_list(src, nmax, count_max,
                                                                          static_cast<uint8_t *>(scr), scr_bytes, st,
                                                                          c.num_cus);
        case BI_MUL_NTT:
            return launch_bigmul_ntt_list(c.ntt.c, src, nmax, count_max, static_cast<uint32_t *>(scr), st, c.num_cus);
        case BI_MUL_NTT_PF64:
            return launch_bigmul_ntt64_list(c.ntt.c64, src, nmax, count_max, static_cast<uint64_t *>(scr), st,
                                            c.num_cus);
        case BI_MUL_KARATSUBA:
            return launch_bigmul_kara_list(c, tune, src, nmax, count_max, static_cast<uint8_t *>(scr), scr_bytes, st);
        default: return launch_bigmul_valu_list(src, nmax, count_max, valu_plan_tuned(nmax, tune), st, c.num_cus);
    }
}

// The list kernel of size class k's algorithm (the tuned one, or `algo` when
// it is forced and supports the class) over at most count_max instances.
static hipError_t launch_class(const Ctx &c, const Tune &tune, const ListInst &src, uint32_t k, uint64_t count_max,
                               int algo, void *scr, hipStream_t st) {
    const uint32_t nmax = class_nmax(k);
    int alg = tune.list_algo[k];
    if (algo != BI_MUL_AUTO && algo_supports(algo, nmax)) alg = algo;
    return launch_bigmul_list_algo(c, tune, src, nmax, count_max, alg, scr, class_scratch_bytes(count_max), st);
}

hipError_t launch_bigmul_v_binned(const Ctx &c, const Tune &tune, const void *a, const void *b, void *out,
                                  const bi_desc *desc, const uint32_t *lists, const uint32_t *counts,
                                  const uint32_t *host_counts, uint32_t limb_bits, int algo, void *scratch,
                                  hipStream_t st) {
    const uint32_t wpl = limb_bits / 32;
    auto A = static_cast<const uint32_t *>(a);
    auto B = static_cast<const uint32_t *>(b);
    auto C = static_cast<uint32_t *>(out);
    uint64_t off = 0;
    for (uint32_t k = 0; k < kNumClasses; ++k) {
        const uint64_t n = host_counts[k];
        if (n == 0) continue;
        const ListInst src{A, B, C, desc, lists + off, counts + k, wpl};
        const hipError_t e = launch_class(c, tune, src, k, n, algo, scratch, st);
        if (e != hipSuccess) return e;
        off += n;
    }
    return hipSuccess;
}

hipError_t launch_bigmul_v_core(const Ctx &c, const Tune &tune, const void *a, const void *b, void *out,
                                const bi_desc *desc, uint64_t count_max, const uint64_t *count_ptr,
                                uint32_t limb_bits, int algo, void *scratch, hipStream_t st) {
    uint32_t *counts = static_cast<uint32_t *>(scratch);
    uint32_t *lists = reinterpret_cast<uint32_t *>(static_cast<char *>(scratch) + 256);
    void *cls_scr = static_cast<char *>(scratch) + 256 + lists_bytes(count_max);
    const uint32_t wpl = limb_bits / 32;
    hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(64), 0, st, counts, uint32_t(kNumClasses));
    const uint64_t bins = (count_max + 255) / 256;
    hipLaunchKernelGGL(bin_kernel, dim3(uint32_t(bins < 4096 ? bins : 4096)), dim3(256), 0, st, desc, count_max,
                       count_ptr, wpl, counts, lists, count_max);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    auto A = static_cast<const uint32_t *>(a);
    auto B = static_cast<const uint32_t *>(b);
    auto C = static_cast<uint32_t *>(out);
    for (uint32_t k = 0; k < kNumClasses; ++k) {
        const ListInst src{A, B, C, desc, lists + uint64_t(k) * count_max, counts + k, wpl};
        e = launch_class(c, tune, src, k, count_max, algo, cls_scr, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

bi_status dispatch_bigmul_v(Ctx &c, const void *a, const void *b, void *out, const bi_desc *desc, uint64_t count,
                            uint32_t limb_bits, int algo, hipStream_t st) {
    if (count > 0xFFFFFFFFull) return set_error(BI_ESIZE, "bigmul_v supports up to 2^32-1 descriptors");
    void *scr = nullptr;
    bi_status s = ctx_scratch(c, batch_scratch_bytes(count, c.num_cus), st, &scr);
    if (s != BI_OK) return s;
    hipError_t e = launch_bigmul_v_core(c, c.tune, a, b, out, desc, count, nullptr, limb_bits, algo, scr, st);
    if (e != hipSuccess) return set_error(BI_EHIP, "bigmul_v launch: %s", hipGetErrorString(e));
    return BI_OK;
}

}  // namespace bi
