// Shared device helpers for the gfx950 kernels: wavefront ballots and the
// carry-lookahead "ballot adder" used by every carry-propagation step.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bi {

constexpr int kWave = 64;  // CDNA wavefront width

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Index of the calling wavefront within the workgroup, marked wave-uniform so
// that everything derived from it lives in SGPRs (scalar loads, scalar loops).
__device__ __forceinline__ uint32_t wave_in_block() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Global wavefront index (uniform).
__device__ __forceinline__ uint64_t wave_global() {
    return uint64_t(blockIdx.x) * (blockDim.x >> 6) + wave_in_block();
}

// Carry propagation over 64 consecutive chunks held one per lane.
//
// Section 2 derives the carry of every limb from an exclusive scan whose
// operator combines (overflow, all-ones) pairs.  Over one wavefront the same
// carries come out of one 64-bit integer addition of the ballot masks:
// with G = generate mask (the chunk overflowed on its own) and P = propagate
// mask (the chunk sum is all-ones; G and P are disjoint), adding X = G | P and
// Y = G with carry-in cin gives S = X + Y + cin, whose internal bit carries are
// exactly the chunk carries: carry into lane i = bit i of (S ^ X ^ Y) =
// bit i of (S ^ P).  The carry out of the 64-bit addition is the carry out of
// lane 63.
struct WaveCarry {
    uint64_t into;  // bit i: carry into lane i
    uint32_t out;   // carry out of lane 63 (0/1)
};

__device__ __forceinline__ WaveCarry wave_carry(uint64_t G, uint64_t P, uint32_t cin) {
    const uint64_t X = G | P;
    const uint64_t t = X + G;
    const uint32_t c1 = t < X;
    const uint64_t S = t + (uint64_t)cin;
    const uint32_t c2 = S < t;
    WaveCarry r;
    r.into = S ^ P;
    r.out = c1 | c2;
    return r;
}

// Add a 0/1 carry into a little-endian run of W 32-bit words.
template <int W>
__device__ __forceinline__ void add_carry_words(uint32_t (&s)[W], uint32_t c) {
#pragma unroll
    for (int w = 0; w < W; ++w) {
        uint32_t co;
        s[w] = __builtin_addc(s[w], 0u, c, &co);
        c = co;
    }
}

// s = x + y over W words; returns the carry out.
template <int W>
__device__ __forceinline__ uint32_t add_words(const uint32_t (&x)[W], const uint32_t (&y)[W], uint32_t (&s)[W]) {
    uint32_t c = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        uint32_t co;
        s[w] = __builtin_addc(x[w], y[w], c, &co);
        c = co;
    }
    return c;
}

template <int W>
__device__ __forceinline__ bool all_ones(const uint32_t (&s)[W]) {
    uint32_t v = 0xFFFFFFFFu;
#pragma unroll
    for (int w = 0; w < W; ++w) v &= s[w];
    return v == 0xFFFFFFFFu;
}

// Vector load/store of W consecutive 32-bit words (W = 1, 2, 4), naturally
// aligned.  NT marks the access non-temporal (streamed data that is touched
// once), which keeps it from displacing other lines in the caches.
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <int W, bool NT = false>
__device__ __forceinline__ void load_words(const uint32_t *p, uint32_t (&v)[W]) {
    if constexpr (W == 1) {
        v[0] = NT ? __builtin_nontemporal_load(p) : *p;
    } else if constexpr (W == 2) {
        const u32x2 *q = reinterpret_cast<const u32x2 *>(p);
        const u32x2 t = NT ? __builtin_nontemporal_load(q) : *q;
        v[0] = t.x; v[1] = t.y;
    } else {
        const u32x4 *q = reinterpret_cast<const u32x4 *>(p);
        const u32x4 t = NT ? __builtin_nontemporal_load(q) : *q;
        v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
    }
}

template <int W, bool NT = false>
__device__ __forceinline__ void store_words(uint32_t *p, const uint32_t (&v)[W]) {
    if constexpr (W == 1) {
        if (NT) __builtin_nontemporal_store(v[0], p); else *p = v[0];
    } else if constexpr (W == 2) {
        const u32x2 t = {v[0], v[1]};
        u32x2 *q = reinterpret_cast<u32x2 *>(p);
        if (NT) __builtin_nontemporal_store(t, q); else *q = t;
    } else {
        const u32x4 t = {v[0], v[1], v[2], v[3]};
        u32x4 *q = reinterpret_cast<u32x4 *>(p);
        if (NT) __builtin_nontemporal_store(t, q); else *q = t;
    }
}

}  // namespace bi
