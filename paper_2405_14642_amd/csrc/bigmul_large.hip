// Full product of ONE pair of integers longer than the batched kernels take
// (more than 2^18 bits): the paper runs such sizes on slower fall-back
// versions (Section 5.1); here the fall-back is built from the fast batched
// path.  Both operands are cut into k blocks of bw 32-bit words (2^16, 2^17
// or 2^18 bits, the last block zero-padded), the k^2 block products run as
// one ragged batch through the per-size-class kernels (the tuned algorithm
// of the block's size class), and
//     out = sum_{i,j} P_ij 2^(32 bw (i + j))
// is formed by a column-sum kernel, a thread per output word w adding the
// words of every block product that covers w (at most 2k, read once each)
// into 64 bits, split into a low word L[w] and a high word H[w + 1], and
// finally out = L + H by the multi-workgroup addition.  Work grows as k^2
// block products; a four-step NTT across workgroups would grow as
// n log n instead.
#include <algorithm>

#include "bi_common.hpp"
#include "bi_internal.hpp"

namespace bi {

namespace {


// dst = src (n words) followed by zeros up to m words.
__global__ void pad_copy_kernel(uint32_t *__restrict__ dst, const uint32_t *__restrict__ src, uint64_t n, uint64_t m) {
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < m; i += uint64_t(gridDim.x) * blockDim.x)
        dst[i] = i < n ? src[i] : 0u;
}

// Descriptor p = i k + j: block i of a times block j of b into product slot p.
__global__ void block_desc_kernel(bi_desc *desc, uint32_t k, uint32_t bw) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= k * k) return;
    const uint32_t i = p / k, j = p - i * k;
    bi_desc d;
    d.a_off = uint64_t(i) * bw;
    d.b_off = uint64_t(j) * bw;
    d.out_off = uint64_t(p) * 2 * bw;
    d.n_limbs = bw;
    d.reserved = 0;
    desc[p] = d;
}

// acc_w = sum of word w - d B of P_ij over i + j = d (low halves, d = w / B)
// and i + j = d - 1 (high halves); L[w] = low word, H[w + 1] = high word.
__global__ void block_fold_kernel(const uint32_t *__restrict__ P, uint32_t *__restrict__ L, uint32_t *__restrict__ H,
                                  uint32_t k, uint32_t bw, uint64_t nout) {
    for (uint64_t w = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; w < nout;
         w += uint64_t(gridDim.x) * blockDim.x) {
        const uint64_t d0 = w / bw;
        uint64_t acc = 0;
        for (uint64_t h = 0; h < 2; ++h) {  // h = 0: low halves at diagonal d0; h = 1: high halves at d0 - 1
            if (h > d0) break;
            const uint64_t d = d0 - h;
            if (d > 2ull * (k - 1)) continue;
            const uint64_t off = w - d * bw;  // in [0, 2 bw)
            const uint64_t i0 = d >= k ? d - (k - 1) : 0, i1 = std::min<uint64_t>(d, k - 1);
            for (uint64_t i = i0; i <= i1; ++i) {
                const uint64_t p = i * k + (d - i);
                acc += P[p * 2 * bw + off];
            }
        }
        L[w] = uint32_t(acc);
        if (w + 1 < nout) H[w + 1] = uint32_t(acc >> 32);
        if (w == 0) H[0] = 0;
    }
}

struct LargeMulLayout {
    uint32_t k, bw;
    uint64_t words;  // k B: padded operand length
    size_t desc, a, b, prod, l, h, vscr, ascr, total;
};

LargeMulLayout large_mul_layout(uint64_t n32, uint32_t bw, int num_cus) {
    LargeMulLayout s;
    s.bw = bw;
    s.k = uint32_t((n32 + bw - 1) / bw);
    s.words = uint64_t(s.k) * bw;
    const uint64_t kk = uint64_t(s.k) * s.k, nout = 2 * n32;
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    s.desc = 0;
    s.a = al(s.desc + kk * sizeof(bi_desc));
    s.b = al(s.a + 4 * s.words);
    s.prod = al(s.b + 4 * s.words);
    s.l = al(s.prod + 4 * kk * 2 * bw);
    s.h = al(s.l + 4 * nout);
    s.vscr = al(s.h + 4 * nout);
    s.ascr = al(s.vscr + batch_scratch_bytes(kk, num_cus));
    // the addition's chunk width depends on out's alignment: size for the narrowest
    s.total = al(s.ascr + large_add_scratch_bytes(large_add_tiles(nout, 1)));
    return s;
}

}  // namespace

size_t large_mul_scratch_bytes(uint64_t n32, uint32_t bw, int num_cus) {
    return large_mul_layout(n32, bw, num_cus).total;
}

// Measured (one pair, tuned block algorithms): 2^16-bit blocks are fastest up
// to 2^20-bit operands (few large blocks leave most CUs idle: 90 vs 138 us at
// 2^19 bits), 2^18-bit blocks from 2^22 bits up (351 vs 539 us at 2^22, 4.1
// vs 7.8 ms at 2^24: larger NTT blocks do less work per word).
uint32_t large_mul_auto_block(uint64_t n32) { return n32 <= (uint64_t(1) << 15) ? 2048u : kMaxLimbs32; }

hipError_t launch_bigmul_large(const Ctx &c, const uint32_t *a, const uint32_t *b, uint32_t *out, uint64_t n32,
                               uint32_t bw, int algo, uint8_t *scratch, hipStream_t st) {
    const LargeMulLayout s = large_mul_layout(n32, bw, c.num_cus);
    const uint64_t kk = uint64_t(s.k) * s.k, nout = 2 * n32;
    auto *desc = reinterpret_cast<bi_desc *>(scratch + s.desc);
    auto *A = reinterpret_cast<uint32_t *>(scratch + s.a);
    auto *B = reinterpret_cast<uint32_t *>(scratch + s.b);
    auto *P = reinterpret_cast<uint32_t *>(scratch + s.prod);
    auto *L = reinterpret_cast<uint32_t *>(scratch + s.l);
    auto *H = reinterpret_cast<uint32_t *>(scratch + s.h);
    const uint32_t cap = uint32_t(c.num_cus) * 16;
    const auto grid = [cap](uint64_t items) { return dim3(uint32_t(std::min<uint64_t>((items + 255) / 256, cap))); };
    hipLaunchKernelGGL(pad_copy_kernel, grid(s.words), dim3(256), 0, st, A, a, n32, s.words);
    hipLaunchKernelGGL(pad_copy_kernel, grid(s.words), dim3(256), 0, st, B, b, n32, s.words);
    hipLaunchKernelGGL(block_desc_kernel, dim3(uint32_t((kk + 255) / 256)), dim3(256), 0, st, desc, s.k, bw);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_bigmul_v_core(c, c.tune, A, B, P, desc, kk, nullptr, 32, algo, scratch + s.vscr, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(block_fold_kernel, grid(nout), dim3(256), 0, st, P, L, H, s.k, bw, nout);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_bigadd_large(L, H, out, nullptr, nout, scratch + s.ascr, st, c.num_cus);
}

}  // namespace bi
