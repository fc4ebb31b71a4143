// Schoolbook multiplication on the VALU (Section 3: eq. (1), the load-balanced
// partition of Fig. 4, the per-thread convolution and combine of Fig. 6, and
// the L/H publication and final addition of Fig. 5), for the full 2n-limb
// product of n-limb operands (32-bit limbs).
//
// gfx950 mapping:
//  * one workgroup per instance; B is staged in LDS between zero pads, A is
//    read with uniform (scalar) loads because every lane of a wave consumes the
//    same A_i at the same step;
//  * a wave computes a block of 64*Q consecutive output coefficients, Q per
//    lane (the paper's sequentialisation factor).  For step i every lane needs
//    B_{k-i} for its Q coefficients; consecutive steps slide that window down by
//    one word, so 4 steps need one 16-byte (Q=4) or two 8-byte (Q=2) LDS reads
//    per lane, conflict-free across the wave;
//  * each product term is one v_mad_u64_u32 into a 64-bit accumulator plus an
//    add-with-carry into a 32-bit overflow counter (the paper's (ubig, uint32)
//    accumulator, Section 3.1);
//  * the loop over i for a block covers the union of the lanes' ranges; terms
//    outside a coefficient's range multiply a zero pad of B (or A = 0 past the
//    operand end), so no lane branches;
//  * blocks differ in cost (a triangle, Fig. 4); waves take them in a snake
//    order over blocks sorted by cost, which balances the waves the same way
//    the paper pairs C_t with C_{M-1-t};
//  * after a barrier the per-thread (Q low words, high word, carry) results
//    are in L and H (compact, 2 words per lane group) and the workgroup adds
//    L + H with the ballot-adder carry scan.
#include "bi_common.hpp"
#include "bi_internal.hpp"
#include "bi_valu.hpp"
#include "bi_wgadd.hpp"

namespace bi {

namespace {

// Zero words on each side of B.  A block spans 64 Q coefficients and the i
// loop runs over 4-aligned groups, so B is indexed from -(64 Q + 3) up to
// n + 64 Q + 1.
template <int Q> constexpr uint32_t pad_words() { return 64 * Q + 4; }

// Block b of the cost-sorted order: 0, NB-1, 1, NB-2, ... (costs rise toward
// the middle of the product, Fig. 4).
__device__ __forceinline__ uint32_t sorted_block(uint32_t idx, uint32_t NB) {
    return (idx & 1u) ? NB - 1 - (idx >> 1) : (idx >> 1);
}

template <int Q>
__device__ __forceinline__ void load_window(const uint32_t *Bsh, int32_t addr, uint32_t (&x)[4]) {
    if constexpr (Q == 4) {
        const uint4 v = *reinterpret_cast<const uint4 *>(Bsh + addr);
        x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
    } else {
        const uint2 v0 = *reinterpret_cast<const uint2 *>(Bsh + addr);
        const uint2 v1 = *reinterpret_cast<const uint2 *>(Bsh + addr + 2);
        x[0] = v0.x; x[1] = v0.y; x[2] = v1.x; x[3] = v1.y;
    }
}

}  // namespace

template <int Q, int NW, class Src>
__global__ __launch_bounds__(64 * NW) void bigmul_valu_kernel(Src src) {
    extern __shared__ __align__(16) uint32_t lds[];
    constexpr uint32_t span = 64 * Q;
    constexpr uint32_t kPad = pad_words<Q>();
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = wave_in_block();
    const uint64_t count = src.count();

    for (uint64_t inst = blockIdx.x; inst < count; inst += gridDim.x) {
        const InstRef in = src.get(inst);
        const uint32_t n = in.n;
        const uint32_t *a = in.a;
        const uint32_t *b = in.b;
        const uint32_t NB = (2 * n + span - 1) / span;  // blocks over the 2n output words
        const uint32_t nbw = (n + 2 * kPad + 3) & ~3u;
        uint32_t *Bsh = lds;                              // [nbw]
        uint32_t *Lsh = Bsh + nbw;                        // [NB * span]
        uint2 *Hsh = reinterpret_cast<uint2 *>(Lsh + NB * span);  // [NB * 64]
        uint32_t *summary = reinterpret_cast<uint32_t *>(Hsh + NB * 64);  // [NW]
        for (uint32_t t = tid; t < nbw; t += 64 * NW) Bsh[t] = (t >= kPad && t < kPad + n) ? b[t - kPad] : 0u;
        __syncthreads();

        for (uint32_t r = 0;; ++r) {
            const uint32_t slot = (r & 1u) ? (NW - 1 - wave) : wave;  // snake
            const uint32_t idx = r * NW + slot;
            if (idx >= NB) break;
            const uint32_t blk = sorted_block(idx, NB);
            const uint32_t k0 = blk * span;
            const uint32_t kl = k0 + Q * lane;
            // union of the lanes' ranges of i, aligned down to a multiple of 4
            const uint32_t ilo = (k0 + 1 > n ? k0 + 1 - n : 0u) & ~3u;
            const uint32_t ihi = min(k0 + span - 1, n - 1);

            uint64_t acc[Q];
            uint32_t cnt[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) { acc[q] = 0; cnt[q] = 0; }

            // Window w[q] = B[kl + q - i] at the current i (B index + kPad = LDS index).
            uint32_t w[4];
            load_window<Q>(Bsh, int32_t(kPad + kl) - int32_t(ilo), w);
            for (uint32_t i = ilo; i <= ihi; i += 4) {
                uint32_t x[4];  // B[kl - i - 4 .. kl - i - 1]
                load_window<Q>(Bsh, int32_t(kPad + kl) - int32_t(i) - 4, x);
                uint32_t av[4];
                if (i + 3 < n) {
#pragma unroll
                    for (int u = 0; u < 4; ++u) av[u] = a[i + u];
                } else {
#pragma unroll
                    for (int u = 0; u < 4; ++u) av[u] = (i + u < n) ? a[i + u] : 0u;
                }
                // step i+u, coefficient q needs B[kl + q - i - u] = cat(x, w)[q - u + 4]
#pragma unroll
                for (int u = 0; u < 4; ++u) {
#pragma unroll
                    for (int q = 0; q < Q; ++q) {
                        const int t = q - u + 4;
                        const uint32_t bv = t >= 4 ? w[t - 4] : x[t];
                        mac(acc[q], cnt[q], av[u], bv);
                    }
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) w[q] = x[q];
            }

            // Combine the Q (accumulator, overflow count) pairs into Q low words,
            // one high word and one carry word (Fig. 6, combine): position p
            // collects lo(acc[p]) + hi(acc[p-1]) + cnt[p-2] and the running carry.
            uint32_t R[Q + 2];
            uint64_t carry = 0;
#pragma unroll
            for (int p = 0; p < Q + 2; ++p) {
                uint64_t s = carry;
                if (p < Q) s += uint32_t(acc[p]);
                if (p >= 1 && p <= Q) s += uint32_t(acc[p - 1] >> 32);
                if (p >= 2) s += cnt[p - 2];
                R[p] = uint32_t(s);
                carry = s >> 32;
            }
#pragma unroll
            for (int q = 0; q < Q; ++q) Lsh[kl + q] = R[q];
            Hsh[blk * 64 + lane] = make_uint2(R[Q], R[Q + 1]);
        }
        __syncthreads();

        // out = L + H over 2n words.  H holds, for lane group g (coefficients
        // Q g .. Q g + Q - 1), its high word at position Q (g+1) and its carry
        // word at Q (g+1) + 1.
        auto lh = [&](uint32_t c, uint32_t (&x)[4], uint32_t (&y)[4]) {
            const uint4 l = *reinterpret_cast<const uint4 *>(Lsh + 4 * c);
            x[0] = l.x; x[1] = l.y; x[2] = l.z; x[3] = l.w;
            if constexpr (Q == 4) {
                if (c >= 1) {
                    const uint2 h = Hsh[c - 1];
                    y[0] = h.x; y[1] = h.y;
                }
            } else {
                if (c >= 1) {
                    const uint2 h = Hsh[2 * c - 1];
                    y[0] = h.x; y[1] = h.y;
                }
                const uint2 h2 = Hsh[2 * c];
                y[2] = h2.x; y[3] = h2.y;
            }
            const uint32_t base = 4 * c;
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (base + t >= 2 * n) { x[t] = 0; y[t] = 0; }
        };
        wg_add_rows<NW>(lh, in.c, 2 * n, summary);
        __syncthreads();
    }
}

size_t valu_lds_bytes(uint32_t n, int Q, int NW) {
    const uint32_t span = 64 * Q;
    const uint32_t NB = (2 * n + span - 1) / span;
    const uint32_t pad = Q == 4 ? pad_words<4>() : pad_words<2>();
    const uint32_t nbw = (n + 2 * pad + 3) & ~3u;
    return 4ull * (nbw + NB * span + 2ull * NB * 64 + NW);
}

template <int Q, int NW, class Src>
static hipError_t launch_q(const Src &src, size_t lds, uint32_t grid, hipStream_t st) {
    static std::atomic<uint64_t> lds_set{0};  // allow up to the whole 160 KiB LDS of a CU
    hipError_t e = lds_limit_once(reinterpret_cast<const void *>(&bigmul_valu_kernel<Q, NW, Src>), lds_set);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((bigmul_valu_kernel<Q, NW, Src>), dim3(grid), dim3(64 * NW), lds, st, src);
    return hipGetLastError();
}

// Configuration for n 32-bit limbs: Q = 2 below 4096 limbs (less work wasted
// at block edges), Q = 4 above (fits LDS at 8192 limbs); waves = number of
// block pairs, capped at 16.
ValuPlan valu_plan(uint32_t n) {
    ValuPlan p;
    p.Q = n > 4096 ? 4 : 2;
    const uint32_t NB = (2 * n + 64 * p.Q - 1) / (64 * p.Q);
    uint32_t nw = (NB + 1) / 2;
    p.NW = nw >= 16 ? 16 : nw >= 8 ? 8 : nw >= 4 ? 4 : nw >= 2 ? 2 : 1;
    p.lds = valu_lds_bytes(n, p.Q, p.NW);
    return p;
}

bool valu_plan_fits(uint32_t n, int Q, int NW, ValuPlan *out) {
    if ((Q != 2 && Q != 4) || (NW != 1 && NW != 2 && NW != 4 && NW != 8 && NW != 16)) return false;
    const size_t lds = valu_lds_bytes(n, Q, NW);
    if (lds > 160 * 1024) return false;
    if (out) *out = ValuPlan{Q, NW, lds};
    return true;
}

ValuPlan valu_plan_tuned(uint32_t n, const Tune &t) {
    const uint32_t k = size_class_host(n);
    ValuPlan p;
    if (t.valu_q[k] && valu_plan_fits(n, t.valu_q[k], t.valu_nw[k], &p)) return p;
    return valu_plan(n);
}

// A plan sized for instances of up to nmax limbs (Q, waves and LDS of the
// largest); smaller instances of a ragged class run with the same plan.
template <class Src>
static hipError_t launch_plan(const Src &src, const ValuPlan &p, uint64_t count, hipStream_t st, int num_cus) {
    const uint64_t cap = uint64_t(num_cus) * 32;
    const uint32_t grid = uint32_t(count < cap ? count : cap);
    if (grid == 0) return hipSuccess;
#define BI_VALU_CASE(QQ, WW) \
    if (p.Q == QQ && p.NW == WW) return launch_q<QQ, WW>(src, p.lds, grid, st);
    BI_VALU_CASE(2, 1) BI_VALU_CASE(2, 2) BI_VALU_CASE(2, 4) BI_VALU_CASE(2, 8) BI_VALU_CASE(2, 16)
    BI_VALU_CASE(4, 1) BI_VALU_CASE(4, 2) BI_VALU_CASE(4, 4) BI_VALU_CASE(4, 8) BI_VALU_CASE(4, 16)
#undef BI_VALU_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_bigmul_valu(const uint32_t *a, const uint32_t *b, uint32_t *c, uint32_t n, uint64_t batch,
                              const ValuPlan &p, hipStream_t st, int num_cus) {
    if (batch == 0) return hipSuccess;
    return launch_plan(UniformInst{a, b, c, n, batch}, p, batch, st, num_cus);
}

hipError_t launch_bigmul_valu_list(const ListInst &src, uint32_t nmax, uint64_t count_max, const ValuPlan &p,
                                   hipStream_t st, int num_cus) {
    (void)nmax;  // p is sized for the class's largest instance
    return launch_plan(src, p, count_max, st, num_cus);
}

}  // namespace bi
