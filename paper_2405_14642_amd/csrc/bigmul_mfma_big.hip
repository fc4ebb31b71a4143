// int8-MFMA schoolbook for products above 1024 limbs (up to 2^18 bits): the
// same block-Toeplitz convolution as bigmul_mfma.hip (eq. (1) of Section 3.1
// on balanced base-256 digits), split so that one product occupies several
// workgroups and its operands no longer need to sit in one workgroup's LDS.
//
//   recode:  per product, the balanced digits of a (natural order, 64 zero
//            bytes before and after) and of b (16-digit groups byte-reversed,
//            the two halves of every 32-digit block in two planes) and the
//            carries t_A, t_B go to a per-product scratch slot.
//   mfma:    per (product, group of 8 supertiles = 256 output blocks), four
//            waves, each owning two adjacent supertiles with accumulators in
//            AGPRs.  The u-range of the group is walked in segments of kSU
//            steps: the segment's digits of a are staged in LDS and expanded
//            into 8-byte windows, the B blocks it needs are copied in (zeros
//            outside the operand), and every wave runs its MFMA steps.  At the
//            end each lane folds its coefficients (plus the t_A / t_B cross
//            terms) into a low word L[w] and a high word H[w + 1] in scratch.
//   carry:   per product, L + H with the workgroup ballot-adder.
#include <algorithm>
#include <atomic>

#include "bi_common.hpp"
#include "bi_internal.hpp"
#include "bi_mfma.hpp"
#include "bi_wgadd.hpp"

namespace bi {

namespace {

using namespace mfma;

constexpr uint32_t kSU = 96;                 // u-steps per segment (LDS < 40 KB: 4 workgroups per CU)
constexpr uint32_t kPadA = 64;               // zero bytes around a's digits in scratch
constexpr uint32_t kNEs = 32 * kSU + 32;     // windows per segment
constexpr uint32_t kStage = 32 * kSU + 48;   // staged digit bytes per segment
constexpr uint32_t kNBS = 255 + kSU;         // B entries per plane and segment
constexpr uint32_t kLdsE8 = 0, kLdsStage = 8 * kNEs, kLdsB = kLdsStage + kStage;
constexpr uint32_t kLdsTotal = kLdsB + 2 * 16 * kNBS;
constexpr int kGroupSt = 8;                  // supertiles per workgroup (4 waves x 2)
constexpr int kNWCarry = 16;

// Byte offsets inside one product's scratch slot (n32p = limbs rounded up to 8).
struct BigSlot {
    uint64_t ad, bp, tt, lh, size;
};

__host__ __device__ inline BigSlot big_slot(uint32_t n32p) {
    const uint64_t D = 4ull * n32p;
    BigSlot s;
    s.ad = 0;                            // D + 2 kPadA bytes
    s.bp = D + 2 * kPadA;                // 2 planes x D/32 entries x 16 bytes
    s.tt = s.bp + D;                     // t_A, t_B (+ padding)
    s.lh = (s.tt + 16 + 255) & ~255ull;  // L (2 n32p words), then H (2 n32p words)
    s.size = (s.lh + 4 * D + 255) & ~255ull;
    return s;
}

template <class Src>
__device__ __forceinline__ uint64_t big_count(const Src &src, uint64_t base, uint64_t chunk) {
    const uint64_t c = src.count();
    return c > base ? min(c - base, chunk) : 0;
}

}  // namespace

// NW waves: one 64-chunk row of each operand per wave at the largest size
// (8 at up to 2^16 bits, 16 above), so no wave idles through the scans.
template <int NW, class Src>
__global__ __launch_bounds__(64 * NW) void mfma_big_recode_kernel(Src src, uint64_t base, uint64_t chunk,
                                                                          uint8_t *__restrict__ scr,
                                                                          uint64_t stride) {
    __shared__ uint32_t summary[2 * NW];
    const uint64_t cnt = big_count(src, base, chunk);
    for (uint64_t q = blockIdx.x; q < cnt; q += gridDim.x) {
        const InstRef in = src.get(base + q);
        const uint32_t n32 = in.n, n32p = (n32 + 7) & ~7u, D = 4 * n32p, nb = D / 32;
        const BigSlot sl = big_slot(n32p);
        uint8_t *slot = scr + q * stride;
        uint8_t *ad = slot + sl.ad;
        uint8_t *bp = slot + sl.bp;
        const uint32_t *a = in.a, *b = in.b;
        auto src_a = [&](uint32_t c, uint32_t (&x)[4], uint32_t (&y)[4]) {
            load4(a, n32, c, x);
            y[0] = y[1] = y[2] = y[3] = kR8;
        };
        auto sink_a = [&](uint32_t c, const uint32_t (&s)[4]) {
            *reinterpret_cast<uint4 *>(ad + kPadA + 16 * c) =
                make_uint4(s[0] ^ kR8, s[1] ^ kR8, s[2] ^ kR8, s[3] ^ kR8);
        };
        const uint32_t tA = wg_add_rows_sink<NW>(src_a, sink_a, n32p, summary);
        auto src_b = [&](uint32_t c, uint32_t (&x)[4], uint32_t (&y)[4]) {
            load4(b, n32, c, x);
            y[0] = y[1] = y[2] = y[3] = kR8;
        };
        auto sink_b = [&](uint32_t c, const uint32_t (&s)[4]) {
            *reinterpret_cast<uint4 *>(bp + (c & 1u) * 16 * nb + 16 * (c >> 1)) =
                make_uint4(__builtin_bswap32(s[3] ^ kR8), __builtin_bswap32(s[2] ^ kR8),
                           __builtin_bswap32(s[1] ^ kR8), __builtin_bswap32(s[0] ^ kR8));
        };
        const uint32_t tB = wg_add_rows_sink<NW>(src_b, sink_b, n32p, summary + NW);
        const uint32_t t = threadIdx.x;
        if (t < 2 * kPadA / 16) {
            const uint32_t off = t < kPadA / 16 ? 16 * t : kPadA + D + 16 * (t - kPadA / 16);
            *reinterpret_cast<uint4 *>(ad + off) = make_uint4(0, 0, 0, 0);
        }
        if (t == 0) {
            uint32_t *tt = reinterpret_cast<uint32_t *>(slot + sl.tt);
            tt[0] = tA;
            tt[1] = tB;
            reinterpret_cast<uint32_t *>(slot + sl.lh)[2 * n32p] = 0;  // H[0]
        }
        __syncthreads();  // summaries are reused by the next product
    }
}

template <class Src>
__global__ __launch_bounds__(256, 4) void mfma_big_kernel(Src src, uint64_t base, uint64_t chunk, uint32_t groups,
                                                       uint8_t *__restrict__ scr, uint64_t stride) {
    extern __shared__ __align__(16) uint8_t lds[];
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = wave_in_block();
    const uint32_t r = lane & 31u, g = lane >> 5;
    const uint64_t cnt = big_count(src, base, chunk);
    uint8_t *e8 = lds + kLdsE8;
    uint8_t *stage = lds + kLdsStage;
    uint8_t *bl = lds + kLdsB;
    for (uint64_t item = blockIdx.x; item < cnt * groups; item += gridDim.x) {
        const uint64_t q = item / groups;
        const uint32_t grp = uint32_t(item - q * groups);
        const InstRef in = src.get(base + q);
        const uint32_t n32p = (in.n + 7) & ~7u, D = 4 * n32p, nb = D / 32;
        const uint32_t nst = (n32p + 127) / 128;
        const uint32_t st0 = kGroupSt * grp;
        if (st0 >= nst) continue;  // uniform across the workgroup
        const uint32_t stl = min(st0 + kGroupSt - 1, nst - 1);
        const BigSlot sl = big_slot(n32p);
        const uint8_t *slot = scr + q * stride;
        const uint8_t *ad = slot + sl.ad;
        const uint8_t *bp = slot + sl.bp;
        const uint32_t *tt = reinterpret_cast<const uint32_t *>(slot + sl.tt);
        const uint32_t tA = tt[0], tB = tt[1];

        // this wave's supertiles (rotated so every SIMD sees every position)
        const uint32_t pw = (wave + uint32_t(item & 3)) & 3u;
        const uint32_t s0 = st0 + 2 * pw, s1 = s0 + 1;
        const bool has0 = s0 <= stl, has1 = s1 <= stl;
        const int32_t lo0 = max(0, int32_t(32 * s0) - int32_t(nb) + 1);
        const int32_t hi0 = has0 ? min(int32_t(nb), int32_t(32 * s0 + 31)) + 1 : lo0;
        const int32_t lo1 = has1 ? max(0, int32_t(32 * s1) - int32_t(nb) + 1) : hi0;
        const int32_t hi1 = has1 ? min(int32_t(nb), int32_t(32 * s1 + 31)) + 1 : hi0;
        const int32_t Ulo = max(0, int32_t(32 * st0) - int32_t(nb) + 1);
        const int32_t Uhi = min(int32_t(nb), int32_t(32 * stl + 31)) + 1;
        v16i acc[2] = {};
        const uint32_t oA = 8 * (r - 16 * g + 17);
        for (int32_t u0 = Ulo; u0 < Uhi; u0 += int32_t(kSU)) {
            const int32_t u1 = min(u0 + int32_t(kSU), Uhi), su = u1 - u0;
            // digits [32 u0 - 32, 32 u1 + 16) of a; window e of the segment
            // starts at digit 32 u0 - 32 + e
            const uint8_t *asrc = ad + kPadA + 32 * (u0 - 1);
            for (uint32_t i = tid; i < uint32_t(2 * su + 3); i += 256)
                *reinterpret_cast<uint4 *>(stage + 16 * i) = reinterpret_cast<const uint4 *>(asrc)[i];
            // B entries of blocks bmin .. bmin + 255 + su - 1 (zero outside [0, nb))
            const int32_t bmin = int32_t(32 * st0) - u1 + 1;
            const uint32_t nbs = 255 + uint32_t(su);
            for (uint32_t i = tid; i < 2 * nbs; i += 256) {
                const uint32_t pl = i >= nbs ? 1u : 0u, e = i - pl * nbs;
                const int32_t blk = bmin + int32_t(e);
                uint4 v = make_uint4(0, 0, 0, 0);
                if (blk >= 0 && blk < int32_t(nb)) v = *reinterpret_cast<const uint4 *>(bp + pl * 16 * nb + 16 * blk);
                *reinterpret_cast<uint4 *>(bl + pl * 16 * kNBS + 16 * e) = v;
            }
            __syncthreads();
            {
                const uint32_t *sw = reinterpret_cast<const uint32_t *>(stage);
                for (uint32_t x2 = tid; x2 < uint32_t(16 * su + 16); x2 += 256) {
                    const uint32_t qq = x2 >> 1, sh = 2 * (x2 & 1u);
                    const uint32_t w0 = sw[qq], w1 = sw[qq + 1], w2 = sw[qq + 2];
                    uint4 v;
                    v.x = __builtin_amdgcn_alignbyte(w1, w0, sh);
                    v.y = __builtin_amdgcn_alignbyte(w2, w1, sh);
                    v.z = __builtin_amdgcn_alignbyte(w1, w0, sh + 1);
                    v.w = __builtin_amdgcn_alignbyte(w2, w1, sh + 1);
                    *reinterpret_cast<uint4 *>(e8 + 16 * x2) = v;
                }
            }
            __syncthreads();
            if (has0) {
                // lane's B entry at segment step 0: block 32 s + r - u0
                const uint8_t *bb0 = bl + g * 16 * kNBS + 16 * (int32_t(32 * s0 + r) - u0 - bmin);
                const uint8_t *bb1 = bb0 + 16 * 32;
                mfma_steps<1>(max(lo0, u0) - u0, min(min(lo1, hi0), u1) - u0, e8, oA, bb0, bb1, acc);
                if (has1) {
                    mfma_steps<3>(max(lo1, u0) - u0, min(hi0, u1) - u0, e8, oA, bb0, bb1, acc);
                    mfma_steps<2>(max(max(hi0, lo1), u0) - u0, min(hi1, u1) - u0, e8, oA, bb0, bb1, acc);
                }
            }
            __syncthreads();  // the next segment overwrites the windows and blocks
        }
        // fold: acc[t][4j + i] is coefficient 32 K + 8 j + 4 g + i, K = 32 s + r
        uint32_t *L = reinterpret_cast<uint32_t *>(const_cast<uint8_t *>(slot) + sl.lh);
        uint32_t *H = L + 2 * n32p;
        const uint32_t W = 2 * n32p;
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            if (!(t == 0 ? has0 : has1)) continue;
            const uint32_t st = s0 + uint32_t(t);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t w = 256 * st + 8 * r + 2 * uint32_t(j) + g;
                int32_t c[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) c[e] = acc[t][4 * j + e];
                if (w >= n32p && w < 2 * n32p && (tA | tB)) {
                    const uint32_t m = w - n32p, cc = m >> 2;
                    const uint32_t aw = *reinterpret_cast<const uint32_t *>(ad + kPadA + 4 * m);
                    const uint32_t bw =
                        *reinterpret_cast<const uint32_t *>(bp + (cc & 1u) * 16 * nb + 16 * (cc >> 1) + 4 * (3 - (m & 3u)));
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        c[e] += int32_t(tA) * sbyte(bw, 3 - e) + int32_t(tB) * sbyte(aw, e);
                }
                uint64_t V = uint64_t(int64_t(c[0])) + (uint64_t(int64_t(c[1])) << 8) +
                             (uint64_t(int64_t(c[2])) << 16) + (uint64_t(int64_t(c[3])) << 24);
                V += (1ull << 63) - (w > 0 ? (1ull << 31) : 0ull);
                if (w < W) L[w] = uint32_t(V);
                if (w + 1 < W) H[w + 1] = uint32_t(V >> 32);
            }
        }
    }
}

template <class Src>
__global__ __launch_bounds__(64 * kNWCarry) void mfma_big_carry_kernel(Src src, uint64_t base, uint64_t chunk,
                                                                        const uint8_t *__restrict__ scr,
                                                                        uint64_t stride) {
    __shared__ uint32_t summary[kNWCarry];
    const uint64_t cnt = big_count(src, base, chunk);
    for (uint64_t q = blockIdx.x; q < cnt; q += gridDim.x) {
        const InstRef in = src.get(base + q);
        const uint32_t n32p = (in.n + 7) & ~7u;
        const uint32_t *L = reinterpret_cast<const uint32_t *>(scr + q * stride + big_slot(n32p).lh);
        wg_add_rows<kNWCarry>(LHSrc{L, L + 2 * n32p, 2 * in.n}, in.c, 2 * in.n, summary);
        __syncthreads();
    }
}

size_t mfma_big_slot_bytes(uint32_t nmax) { return size_t(big_slot((nmax + 7) & ~7u).size); }

template <class Src>
static hipError_t launch_big(const Src &src, uint32_t nmax, uint64_t count_max, uint64_t chunk, uint8_t *scr,
                             hipStream_t st, int num_cus) {
    static std::atomic<int> occ{0};
    static std::atomic<uint64_t> lds_set{0};
    int nblk = occ.load(std::memory_order_relaxed);
    const void *fn = reinterpret_cast<const void *>(&mfma_big_kernel<Src>);
    hipError_t e = lds_limit_once(fn, lds_set);
    if (e != hipSuccess) return e;
    if (nblk == 0) {
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nblk, fn, 256, kLdsTotal);
        if (e != hipSuccess) return e;
        if (nblk < 1) nblk = 1;
        occ.store(nblk, std::memory_order_relaxed);
    }
    const uint32_t n32p = (nmax + 7) & ~7u;
    const uint32_t groups = ((n32p + 127) / 128 + kGroupSt - 1) / kGroupSt;
    const uint64_t stride = mfma_big_slot_bytes(nmax);
    const uint64_t cap = uint64_t(num_cus > 0 ? num_cus : 1) * 2;
    for (uint64_t b = 0; b < count_max; b += chunk) {
        const uint64_t c = std::min(chunk, count_max - b);
        if (n32p <= 2048)
            hipLaunchKernelGGL((mfma_big_recode_kernel<8, Src>), dim3(uint32_t(std::min(c, cap * 8))), dim3(512), 0,
                               st, src, b, chunk, scr, stride);
        else
            hipLaunchKernelGGL((mfma_big_recode_kernel<16, Src>), dim3(uint32_t(std::min(c, cap * 4))), dim3(1024), 0,
                               st, src, b, chunk, scr, stride);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        const uint64_t items = c * groups;
        const uint64_t g2 = std::min(items, uint64_t(nblk) * uint64_t(num_cus > 0 ? num_cus : 1));
        hipLaunchKernelGGL((mfma_big_kernel<Src>), dim3(uint32_t(g2)), dim3(256), kLdsTotal, st, src, b, chunk, groups,
                           scr, stride);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((mfma_big_carry_kernel<Src>), dim3(uint32_t(std::min(c, cap * 4))), dim3(64 * kNWCarry), 0,
                           st, src, b, chunk, scr, stride);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_bigmul_mfma_big(const uint32_t *a, const uint32_t *b, uint32_t *c, uint32_t n32, uint64_t batch,
                                  uint8_t *scr, hipStream_t st, int num_cus, uint64_t round) {
    if (batch == 0) return hipSuccess;
    if (round == 0) return hipErrorInvalidValue;
    return launch_big(UniformInst{a, b, c, n32, batch}, n32, batch, std::min(batch, round), scr, st, num_cus);
}

hipError_t launch_bigmul_mfma_big_list(const ListInst &src, uint32_t nmax, uint64_t count_max, uint8_t *scr,
                                       size_t scr_bytes, hipStream_t st, int num_cus) {
    const uint64_t chunk = scr_bytes / mfma_big_slot_bytes(nmax);
    if (chunk == 0) return hipErrorInvalidValue;
    return launch_big(src, nmax, count_max, chunk, scr, st, num_cus);
}

}  // namespace bi
