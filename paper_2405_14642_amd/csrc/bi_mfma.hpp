// Device helpers shared by the int8-MFMA schoolbook kernels: operand
// loads, the block-Toeplitz MFMA steps over one or two supertiles, and the
// low/high source of the final carry scan.
#pragma once

#include "bi_common.hpp"
#include "bi_internal.hpp"

namespace bi {
namespace mfma {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr uint32_t kR8 = 0x80808080u;

// Low words L[w] and high words H[w] (H[0] = 0), in LDS or global memory.
struct LHSrc {
    const uint32_t *L;
    const uint32_t *H;
    uint32_t nwords;
    __device__ __forceinline__ void operator()(uint32_t c, uint32_t (&x)[4], uint32_t (&y)[4]) const {
        const uint4 l = *reinterpret_cast<const uint4 *>(L + 4 * c);
        const uint4 h = *reinterpret_cast<const uint4 *>(H + 4 * c);
        x[0] = l.x; x[1] = l.y; x[2] = l.z; x[3] = l.w;
        y[0] = h.x; y[1] = h.y; y[2] = h.z; y[3] = h.w;
        const uint32_t base = 4 * c;
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if (base + t >= nwords) { x[t] = 0; y[t] = 0; }
    }
};

__device__ __forceinline__ void load4(const uint32_t *p, uint32_t n, uint32_t c, uint32_t (&x)[4]) {
    const uint32_t base = 4 * c;
    if (base + 4 <= n && (reinterpret_cast<uintptr_t>(p + base) & 15) == 0) {
        const uint4 v = *reinterpret_cast<const uint4 *>(p + base);
        x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
    } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) x[t] = base + t < n ? p[base + t] : 0u;
    }
}

// Byte i of w as a signed digit.
__device__ __forceinline__ int32_t sbyte(uint32_t w, uint32_t i) { return int32_t(w << (24 - 8 * i)) >> 24; }

// A operand of step u for this lane: two 8-byte windows of a's digits, at
// LDS byte offsets oA + 256 u and oA + 256 u + 64 of the window array (8
// bytes per window; consecutive lanes read consecutive windows).  Both
// addresses are laundered so the compiler keeps separate ds_read_b64
// instead of merging pairs into ds_read2_b64, which the LDS serves at half
// the rate.
__device__ __forceinline__ v4i load_a(const uint8_t *lds, uint32_t oA, int32_t u) {
    uint32_t p0 = oA + 256 * uint32_t(u), p1 = p0 + 64;
    asm volatile("" : "+v"(p0));
    asm volatile("" : "+v"(p1));
    const uint64_t x0 = *reinterpret_cast<const uint64_t *>(lds + p0);
    const uint64_t x1 = *reinterpret_cast<const uint64_t *>(lds + p1);
    return v4i{int(uint32_t(x0)), int(uint32_t(x0 >> 32)), int(uint32_t(x1)), int(uint32_t(x1 >> 32))};
}

// The same operand without the laundering: the compiler may read both
// windows with one ds_read2_b64 (half the LDS rate, no address arithmetic),
// for loops bound by instruction issue rather than by LDS bandwidth.
__device__ __forceinline__ v4i load_a_plain(const uint8_t *lds, uint32_t oA, int32_t u) {
    const uint32_t p0 = oA + 256 * uint32_t(u);
    const uint64_t x0 = *reinterpret_cast<const uint64_t *>(lds + p0);
    const uint64_t x1 = *reinterpret_cast<const uint64_t *>(lds + p0 + 64);
    return v4i{int(uint32_t(x0)), int(uint32_t(x0 >> 32)), int(uint32_t(x1)), int(uint32_t(x1 >> 32))};
}

// MFMA steps u in [ua, ub) for supertile s0 (M bit 0) and/or s1 = s0 + 1
// (M bit 1), which share the A operand T_u.  bb0 / bb1: this lane's B entry
// of step 0 for s0 / s1 (the entry of step u is 16 u bytes lower).
// acc[0] accumulates s0, acc[1] s1.
template <int M, bool PLAIN = false>
__device__ __forceinline__ void mfma_steps(int32_t ua, int32_t ub, const uint8_t *lds, uint32_t oA,
                                           const uint8_t *bb0, const uint8_t *bb1, v16i (&acc)[2]) {
    auto ldB = [](const uint8_t *bb, int32_t u) -> v4i { return *reinterpret_cast<const v4i *>(bb - 16 * u); };
    int32_t u = ua;
    for (; u + 1 < ub; u += 2) {
        const v4i a0 = PLAIN ? load_a_plain(lds, oA, u) : load_a(lds, oA, u);
        const v4i a1 = PLAIN ? load_a_plain(lds, oA, u + 1) : load_a(lds, oA, u + 1);
        v4i p0 = {}, p1 = {}, q0 = {}, q1 = {};
        if (M & 1) { p0 = ldB(bb0, u); p1 = ldB(bb0, u + 1); }
        if (M & 2) { q0 = ldB(bb1, u); q1 = ldB(bb1, u + 1); }
        if (M & 1) acc[0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0, p0, acc[0], 0, 0, 0);
        if (M & 2) acc[1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0, q0, acc[1], 0, 0, 0);
        if (M & 1) acc[0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1, p1, acc[0], 0, 0, 0);
        if (M & 2) acc[1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1, q1, acc[1], 0, 0, 0);
    }
    if (u < ub) {
        const v4i a0 = PLAIN ? load_a_plain(lds, oA, u) : load_a(lds, oA, u);
        if (M & 1) acc[0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0, ldB(bb0, u), acc[0], 0, 0, 0);
        if (M & 2) acc[1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0, ldB(bb1, u), acc[1], 0, 0, 0);
    }
}

}  // namespace mfma
}  // namespace bi
