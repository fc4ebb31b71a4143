// Workgroup-cooperative big-integer addition x + y of two little-endian word
// arrays that live in LDS (or are computed on the fly), written to global
// memory.  This is the final step of every multiplication: the paper adds the
// low and high/carry parts published by the threads with the addition of
// Section 2 (Fig. 5, baddRegs); Section 4 does the same after the inverse
// transform.
//
// Layout: a "row" is 64 lanes x 4 words (256 words).  Each wave owns a
// contiguous range of rows.  Pass 1 reduces every wave's range to a summary
// (carry out with carry-in 0, and whether every chunk propagates); after a
// barrier each wave derives its carry-in from the summaries of the waves
// below it, then pass 2 recomputes its rows with that carry-in and stores.
#pragma once

#include "bi_common.hpp"

namespace bi {

// src(c, x, y) fills the 4 words of chunk c (words 4c .. 4c+3) of both
// addends; sink(c, s) receives the 4 sum words of chunk c (only for chunks
// with c < nchunks).  Words at index >= nwords must read as 0.  cin0 (0 or
// 1) is a carry into word 0.  Returns, in every thread, the carry out of the
// whole sum when nwords is a multiple of 4 (otherwise that carry stays inside
// the last chunk's sum words).  Contains barriers: every thread of the
// workgroup must call it.
template <int NW, class Src, class Sink>
__device__ __forceinline__ uint32_t wg_add_rows_sink(const Src &src, const Sink &sink, uint32_t nwords,
                                                     uint32_t *summary /* LDS, NW words */, uint32_t cin0 = 0) {
    const uint32_t lane = lane_id();
    const uint32_t w = wave_in_block();
    const uint32_t nchunks = (nwords + 3) / 4;
    const uint32_t rows = (nchunks + 63) / 64;
    const uint32_t r0 = (rows * w) / NW, r1 = (rows * (w + 1)) / NW;

    // wave 0's summary includes cin0, so the waves above fold it in below
    uint32_t cin = w == 0 ? cin0 : 0, allp = 1;
    for (uint32_t r = r0; r < r1; ++r) {
        const uint32_t c = r * 64 + lane;
        uint32_t x[4] = {0, 0, 0, 0}, y[4] = {0, 0, 0, 0}, s[4];
        if (c < nchunks) src(c, x, y);
        const uint32_t g = add_words<4>(x, y, s);
        const bool p = c < nchunks && all_ones<4>(s);
        const uint64_t G = ballot(g), P = ballot(p);
        const WaveCarry wc = wave_carry(G, P, cin);
        // a partial last row carries out of its first unused lane
        const uint32_t valid = min(nchunks - r * 64, 64u);
        const uint64_t vmask = valid >= 64 ? ~0ull : ((1ull << valid) - 1);
        cin = valid >= 64 ? wc.out : uint32_t(wc.into >> valid) & 1u;
        allp &= (P == vmask) ? 1u : 0u;
    }
    if (lane == 0) summary[w] = cin | (allp << 1);
    __syncthreads();
    cin = 0;
    uint32_t total = 0;
    for (uint32_t v = 0; v < NW; ++v) {
        const uint32_t sv = summary[v];
        if (v < w) cin = (sv & 1u) | ((sv >> 1) & cin);
        total = (sv & 1u) | ((sv >> 1) & total);
    }
    if (w == 0) cin = cin0;
    for (uint32_t r = r0; r < r1; ++r) {
        const uint32_t c = r * 64 + lane;
        uint32_t x[4] = {0, 0, 0, 0}, y[4] = {0, 0, 0, 0}, s[4];
        if (c < nchunks) src(c, x, y);
        const uint32_t g = add_words<4>(x, y, s);
        const bool p = c < nchunks && all_ones<4>(s);
        const uint64_t G = ballot(g), P = ballot(p);
        const WaveCarry wc = wave_carry(G, P, cin);
        const uint32_t ci = uint32_t(wc.into >> lane) & 1u;
        add_carry_words<4>(s, ci);
        const uint32_t valid = min(nchunks - r * 64, 64u);
        cin = valid >= 64 ? wc.out : uint32_t(wc.into >> valid) & 1u;
        if (c < nchunks) sink(c, s);
    }
    return total;
}

// The same addition with the addends already in registers: wave w owns rows
// w R .. w R + R - 1 (row r = chunks 64 r .. 64 r + 63), and lane l holds
// x[i], y[i] for chunk 64 (w R + i) + l (zero at or beyond nwords).  The
// chunk sums stay in registers between the two halves, so there is one
// barrier and no recomputation; NW R rows must cover nwords.  cin0 (0 or 1)
// is a carry into word 0.  Returns the carry out of the whole sum when
// nwords is a multiple of 4.  Every thread of the workgroup must call it.
template <int NW, int R, class Sink>
__device__ __forceinline__ uint32_t wg_add_regs(const uint32_t (&x)[R][4], const uint32_t (&y)[R][4],
                                                uint32_t nwords, const Sink &sink, uint32_t *summary /* NW words */,
                                                uint32_t cin0 = 0) {
    const uint32_t lane = lane_id();
    const uint32_t w = wave_in_block();
    const uint32_t nchunks = (nwords + 3) / 4;
    uint32_t s[R][4];
    uint64_t G[R], P[R];
    uint32_t valid[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const uint32_t r = w * R + uint32_t(i);
        const uint32_t c = 64 * r + lane;
        valid[i] = nchunks > 64 * r ? min(nchunks - 64 * r, 64u) : 0u;
        const uint32_t g = add_words<4>(x[i], y[i], s[i]);
        G[i] = ballot(c < nchunks && g);
        P[i] = ballot(c < nchunks && all_ones<4>(s[i]));
    }
    // carry out of this wave's rows with carry-in 0 (cin0 for wave 0), and
    // whether every valid chunk propagates
    uint32_t cin = w == 0 ? cin0 : 0, allp = 1;
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const WaveCarry wc = wave_carry(G[i], P[i], cin);
        const uint32_t v = valid[i];
        const uint64_t vmask = v >= 64 ? ~0ull : ((1ull << v) - 1);
        cin = v >= 64 ? wc.out : uint32_t(wc.into >> v) & 1u;
        allp &= (P[i] == vmask) ? 1u : 0u;
    }
    if (lane == 0) summary[w] = cin | (allp << 1);
    __syncthreads();
    cin = 0;
    uint32_t total = 0;
    for (uint32_t v = 0; v < uint32_t(NW); ++v) {
        const uint32_t sv = summary[v];
        if (v < w) cin = (sv & 1u) | ((sv >> 1) & cin);
        total = (sv & 1u) | ((sv >> 1) & total);
    }
    if (w == 0) cin = cin0;
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const uint32_t c = 64 * (w * R + uint32_t(i)) + lane;
        const WaveCarry wc = wave_carry(G[i], P[i], cin);
        add_carry_words<4>(s[i], uint32_t(wc.into >> lane) & 1u);
        const uint32_t v = valid[i];
        cin = v >= 64 ? wc.out : uint32_t(wc.into >> v) & 1u;
        if (c < nchunks) sink(c, s[i]);
    }
    return total;
}

// Global-memory sink for wg_add_rows: words >= nwords are dropped.
struct GlobalSink {
    uint32_t *out;
    uint32_t nwords;
    bool vec_ok;
    __device__ __forceinline__ void operator()(uint32_t c, const uint32_t (&s)[4]) const {
        const uint32_t base = 4 * c;
        if (vec_ok && base + 4 <= nwords) {
            store_words<4>(out + base, s);
        } else {
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (base + t < nwords) out[base + t] = s[t];
        }
    }
};

// x + y written to global memory (nwords words).
template <int NW, class Src>
__device__ __forceinline__ void wg_add_rows(const Src &src, uint32_t *__restrict__ out, uint32_t nwords,
                                            uint32_t *summary /* LDS, NW words */) {
    const GlobalSink sink{out, nwords, (reinterpret_cast<uintptr_t>(out) & 15) == 0};
    (void)wg_add_rows_sink<NW>(src, sink, nwords, summary);
}

// Addends of a product in "low / high" form with groups of 4 words: L holds
// the 4 low words of every group at their positions, H[g] the high word and
// carry word of group g, which belong at word positions 4 (g+1) and 4 (g+1)+1.
struct LHSrc4 {
    const uint32_t *L;  // LDS, 4 * ngroups words
    const uint2 *H;     // LDS, ngroups entries
    uint32_t nwords;
    __device__ __forceinline__ void operator()(uint32_t c, uint32_t (&x)[4], uint32_t (&y)[4]) const {
        const uint4 l = *reinterpret_cast<const uint4 *>(L + 4 * c);
        x[0] = l.x; x[1] = l.y; x[2] = l.z; x[3] = l.w;
        if (c >= 1) {
            const uint2 h = H[c - 1];
            y[0] = h.x; y[1] = h.y;
        }
        const uint32_t base = 4 * c;
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if (base + t >= nwords) { x[t] = 0; y[t] = 0; }
    }
};

}  // namespace bi
