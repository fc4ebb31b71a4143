// Batched big-integer addition (Section 2, Fig. 2: bbadd = map badd).
//
// Addition is byte-width agnostic: a little-endian integer of n limbs of w
// bits is the same byte string whatever w is, so the kernels work on "chunks"
// of W 32-bit words (W = 4, 2 or 1; 16, 8 or 4 bytes), one chunk per lane.
// A chunk is the paper's efficient-sequentialisation unit (Q consecutive
// limbs per thread): the lane adds its chunk sequentially with carry-in 0 and
// reduces it to a generate bit (the chunk sum overflowed) and a propagate bit
// (the chunk sum is all-ones), which never hold together.  The carries across
// the 64 chunks of a wavefront "row" then come out of one 64-bit addition of
// the ballot masks (bi::wave_carry); a final map adds the carry into the chunk.
//
// Two schedules, both with one wavefront per independent piece of work and no
// LDS or barriers at all:
//  * packed rows (an instance has m <= 64 chunks): a row holds
//    ipr = floor(64/m) whole instances.  The segmented scan of Fig. 2 becomes
//    masking: generate/propagate bits of the last chunk of every instance are
//    cleared, so no carry crosses an instance boundary and each instance starts
//    with carry-in 0.  (Clearing them is what makes the exclusive segmented
//    scan correct at segment starts.)
//  * streamed rows (m > 64): one wavefront walks an instance from the least
//    significant row upward, carrying the scalar carry-out of each row into the
//    next.  Loads of U rows are issued before any of them is consumed.
#include "bi_common.hpp"
#include "bi_internal.hpp"

namespace bi {

template <int W, int U, bool NT>
__global__ __launch_bounds__(256) void bigadd_packed_kernel(const uint32_t *__restrict__ a,
                                                            const uint32_t *__restrict__ b,
                                                            uint32_t *out, uint8_t *carry,
                                                            uint32_t m, uint32_t ipr, uint64_t batch) {
    const uint32_t lane = lane_id();
    const uint64_t wave = wave_global();
    const uint64_t nwaves = (uint64_t(gridDim.x) * blockDim.x) >> 6;
    const uint32_t slot = lane / m;           // instance within the row
    const uint32_t pos = lane - slot * m;     // chunk within the instance
    const bool in_row = slot < ipr;
    const uint64_t E = ballot(in_row && pos == m - 1);  // last chunk of each instance
    const uint64_t nrows = (batch + ipr - 1) / ipr;

    for (uint64_t r0 = wave * U; r0 < nrows; r0 += nwaves * U) {
        uint32_t va[U][W], vb[U][W];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t inst = (r0 + u) * ipr + slot;
            ok[u] = in_row && (r0 + u) < nrows && inst < batch;
            if (ok[u]) {
                const uint64_t off = (inst * m + pos) * W;
                load_words<W, NT>(a + off, va[u]);
                load_words<W, NT>(b + off, vb[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            uint32_t s[W];
            const uint32_t g = add_words<W>(va[u], vb[u], s);
            const bool p = all_ones<W>(s);
            const uint64_t G = ballot(ok[u] && g) & ~E;
            const uint64_t P = ballot(ok[u] && p) & ~E;
            const WaveCarry wc = wave_carry(G, P, 0u);
            const uint32_t cin = uint32_t(wc.into >> lane) & 1u;
            if (ok[u]) {
                const uint64_t inst = (r0 + u) * ipr + slot;
                if (carry && pos == m - 1) carry[inst] = uint8_t(g | (p & cin));
                add_carry_words<W>(s, cin);
                store_words<W, NT>(out + (inst * m + pos) * W, s);
            }
        }
    }
}

// One wavefront adds one instance of m chunks, least significant row first.
// Returns (in every lane) the carry out of the instance.
template <int W, int U, bool NT>
__device__ __forceinline__ uint32_t add_instance_streamed(const uint32_t *__restrict__ ai,
                                                          const uint32_t *__restrict__ bi_, uint32_t *oi,
                                                          uint32_t m, uint32_t lane) {
    const uint32_t rows = (m + 63) / 64;
    uint32_t cin_row = 0;
    for (uint32_t r0 = 0; r0 < rows; r0 += U) {
        uint32_t va[U][W], vb[U][W];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t c = (r0 + u) * 64 + lane;
            if (c < m) {
                load_words<W>(ai + uint64_t(c) * W, va[u]);
                load_words<W>(bi_ + uint64_t(c) * W, vb[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (r0 + u < rows) {  // uniform
                const uint32_t c = (r0 + u) * 64 + lane;
                const bool ok = c < m;
                uint32_t s[W];
                const uint32_t g = add_words<W>(va[u], vb[u], s);
                const bool p = all_ones<W>(s);
                const uint64_t G = ballot(ok && g);
                const uint64_t P = ballot(ok && p);
                const WaveCarry wc = wave_carry(G, P, cin_row);
                const uint32_t cin = uint32_t(wc.into >> lane) & 1u;
                if (ok) {
                    add_carry_words<W>(s, cin);
                    store_words<W>(oi + uint64_t(c) * W, s);
                }
                // Carry out of this row: out of lane 63 for a full row,
                // otherwise the carry into the first unused lane.
                const uint32_t valid = m - (r0 + u) * 64;
                cin_row = valid >= 64 ? wc.out : uint32_t(wc.into >> valid) & 1u;
            }
        }
    }
    return cin_row;
}

// Ragged batch: one wavefront per descriptor, chunks of one limb (W words).
template <int W, int U>
__global__ __launch_bounds__(256) void bigadd_ragged_kernel(const uint32_t *__restrict__ a,
                                                            const uint32_t *__restrict__ b,
                                                            uint32_t *out, uint8_t *carry,
                                                            const bi_desc *__restrict__ desc, uint64_t count) {
    const uint32_t lane = lane_id();
    const uint64_t wave = wave_global();
    const uint64_t nwaves = (uint64_t(gridDim.x) * blockDim.x) >> 6;
    for (uint64_t i = wave; i < count; i += nwaves) {
        const bi_desc d = desc[i];
        const uint32_t c = add_instance_streamed<W, U, false>(a + d.a_off * W, b + d.b_off * W, out + d.out_off * W,
                                                       d.n_limbs, lane);
        if (carry && lane == 0) carry[i] = uint8_t(c);
    }
}

// Workgroup-cooperative schedule for instances longer than one row: the NW
// waves of a workgroup load disjoint runs of U rows of the same instance at
// once (NW*U rows per tile), reduce each run to a carry summary (carry out
// with carry-in 0, and whether every chunk propagates), exchange the
// summaries through LDS, and then apply their true carry-in.  This is the
// thread -> wave -> block hierarchy of the paper's block scan, with one
// ballot-adder step per level.
template <int W, int U, int NW, bool NT>
__global__ __launch_bounds__(64 * NW) void bigadd_coop_kernel(const uint32_t *__restrict__ a,
                                                              const uint32_t *__restrict__ b,
                                                              uint32_t *out, uint8_t *carry, uint32_t m,
                                                              uint64_t batch) {
    __shared__ uint32_t summ[NW];
    const uint32_t lane = lane_id();
    const uint32_t wave = wave_in_block();
    const uint32_t rows = (m + 63) / 64;
    const uint32_t tiles = (rows + NW * U - 1) / (NW * U);

    for (uint64_t inst = blockIdx.x; inst < batch; inst += gridDim.x) {
        const uint64_t off = inst * m * W;
        const uint32_t *ai = a + off;
        const uint32_t *bi_ = b + off;
        uint32_t *oi = out + off;
        uint32_t tile_cin = 0;
        for (uint32_t tile = 0; tile < tiles; ++tile) {
            const uint32_t r0 = (tile * NW + wave) * U;
            uint32_t s[U][W];
            uint64_t G[U], P[U];
            uint32_t gl[U], pl[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t c = (r0 + u) * 64 + lane;
                uint32_t va[W], vb[W];
#pragma unroll
                for (int w = 0; w < W; ++w) { va[w] = 0; vb[w] = 0; }
                if (c < m) {
                    load_words<W, NT>(ai + uint64_t(c) * W, va);
                    load_words<W, NT>(bi_ + uint64_t(c) * W, vb);
                }
                gl[u] = add_words<W>(va, vb, s[u]);
                pl[u] = (c < m && all_ones<W>(s[u])) ? 1u : 0u;
            }
            // Summary of this wave's run (rows past the instance end are the
            // identity: they neither kill nor generate).
            uint32_t cout = 0, allp = 1;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                G[u] = ballot(gl[u] != 0);
                P[u] = ballot(pl[u] != 0);
                if (r0 + u < rows) {  // uniform
                    const uint32_t valid = min(m - (r0 + u) * 64, 64u);
                    const uint64_t vmask = valid >= 64 ? ~0ull : ((1ull << valid) - 1);
                    const WaveCarry wc = wave_carry(G[u], P[u], cout);
                    cout = valid >= 64 ? wc.out : uint32_t(wc.into >> valid) & 1u;
                    allp &= (P[u] == vmask) ? 1u : 0u;
                }
            }
            if (lane == 0) summ[wave] = cout | (allp << 1);
            __syncthreads();
            uint32_t cin = tile_cin, tcout = tile_cin;
#pragma unroll
            for (int v = 0; v < NW; ++v) {
                const uint32_t sv = summ[v];
                if (v < int(wave)) cin = (sv & 1u) | ((sv >> 1) & cin);
                tcout = (sv & 1u) | ((sv >> 1) & tcout);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (r0 + u < rows) {  // uniform
                    const uint32_t c = (r0 + u) * 64 + lane;
                    const uint32_t valid = min(m - (r0 + u) * 64, 64u);
                    const WaveCarry wc = wave_carry(G[u], P[u], cin);
                    const uint32_t ci = uint32_t(wc.into >> lane) & 1u;
                    add_carry_words<W>(s[u], ci);
                    if (c < m) store_words<W, NT>(oi + uint64_t(c) * W, s[u]);
                    cin = valid >= 64 ? wc.out : uint32_t(wc.into >> valid) & 1u;
                }
            }
            tile_cin = tcout;
            __syncthreads();  // summ is rewritten by the next tile
        }
        if (carry && threadIdx.x == 0) carry[inst] = uint8_t(tile_cin);
    }
}

// Barrier-free schedule for instances of RPI rows (2 to 8): one wavefront
// loads U whole instances (U * RPI rows) before consuming any, then chains
// the scalar carry through each instance's rows.
template <int W, int U, int RPI, bool NT>
__global__ __launch_bounds__(256) void bigadd_multi_kernel(const uint32_t *__restrict__ a,
                                                           const uint32_t *__restrict__ b,
                                                           uint32_t *out, uint8_t *carry, uint32_t m,
                                                           uint64_t batch) {
    const uint32_t lane = lane_id();
    const uint64_t wave = wave_global();
    const uint64_t nwaves = (uint64_t(gridDim.x) * blockDim.x) >> 6;
    for (uint64_t i0 = wave * U; i0 < batch; i0 += nwaves * U) {
        uint32_t s[U][RPI][W];
        uint32_t gl[U][RPI], pl[U][RPI];
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int r = 0; r < RPI; ++r) {
                const uint32_t c = r * 64 + lane;
                uint32_t va[W], vb[W];
#pragma unroll
                for (int w = 0; w < W; ++w) { va[w] = 0; vb[w] = 0; }
                const bool ok = (i0 + u < batch) && c < m;
                if (ok) {
                    const uint64_t off = ((i0 + u) * m + c) * W;
                    load_words<W, NT>(a + off, va);
                    load_words<W, NT>(b + off, vb);
                }
                gl[u][r] = add_words<W>(va, vb, s[u][r]);
                pl[u][r] = (ok && all_ones<W>(s[u][r])) ? 1u : 0u;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (i0 + u >= batch) break;  // uniform
            uint32_t cin = 0;
#pragma unroll
            for (int r = 0; r < RPI; ++r) {
                const uint32_t c = r * 64 + lane;
                if (r * 64 >= int(m)) break;  // uniform
                const uint64_t G = ballot(gl[u][r] != 0), P = ballot(pl[u][r] != 0);
                const WaveCarry wc = wave_carry(G, P, cin);
                const uint32_t ci = uint32_t(wc.into >> lane) & 1u;
                add_carry_words<W>(s[u][r], ci);
                if (c < m) store_words<W, NT>(out + ((i0 + u) * m + c) * W, s[u][r]);
                const uint32_t valid = min(m - r * 64, 64u);
                cin = valid >= 64 ? wc.out : uint32_t(wc.into >> valid) & 1u;
            }
            if (carry && lane == 0) carry[i0 + u] = uint8_t(cin);
        }
    }
}

// Largest chunk (in bytes) that divides the instance length and all pointers.
static int pick_chunk_bytes(uint64_t inst_bytes, const void *a, const void *b, const void *o) {
    const uint64_t al = uint64_t(reinterpret_cast<uintptr_t>(a)) | uint64_t(reinterpret_cast<uintptr_t>(b)) |
                        uint64_t(reinterpret_cast<uintptr_t>(o)) | inst_bytes;
    if ((al & 15) == 0) return 16;
    if ((al & 7) == 0) return 8;
    return 4;
}

template <int W, int U, bool NT>
static hipError_t launch_wu(const uint32_t *a, const uint32_t *b, uint32_t *o, uint8_t *carry, uint64_t m,
                            uint64_t batch, hipStream_t st, uint64_t max_waves, bool multi) {
    if (m <= 64) {
        const uint32_t ipr = uint32_t(64 / m);
        const uint64_t nrows = (batch + ipr - 1) / ipr;
        uint64_t waves = (nrows + U - 1) / U;
        if (waves > max_waves) waves = max_waves;
        const uint64_t blocks = (waves + 3) / 4;
        hipLaunchKernelGGL((bigadd_packed_kernel<W, U, NT>), dim3(uint32_t(blocks)), dim3(256), 0, st, a, b, o, carry,
                           uint32_t(m), ipr, batch);
    } else if (multi && m <= 8 * 64) {
        // Up to 8 rows: one wave per instance, `U` instances in flight.
        const uint64_t rows = (m + 63) / 64;
        uint64_t waves = (batch + U - 1) / U;
        if (waves > max_waves) waves = max_waves;
        const dim3 g{uint32_t((waves + 3) / 4), 1, 1};
        if (rows <= 2)
            hipLaunchKernelGGL((bigadd_multi_kernel<W, (U > 2 ? U / 2 : 1), 2, NT>), g, dim3(256), 0, st, a, b, o,
                               carry, uint32_t(m), batch);
        else if (rows <= 4)
            hipLaunchKernelGGL((bigadd_multi_kernel<W, (U > 4 ? U / 4 : 1), 4, NT>), g, dim3(256), 0, st, a, b, o,
                               carry, uint32_t(m), batch);
        else
            hipLaunchKernelGGL((bigadd_multi_kernel<W, 1, 8, NT>), g, dim3(256), 0, st, a, b, o, carry, uint32_t(m),
                               batch);
    } else {
        // One workgroup per instance: NW waves x UC rows cover the instance
        // in one tile when it has at most 32 rows.
        const uint64_t rows = (m + 63) / 64;
        uint64_t wgs = batch;
        const uint64_t cap = max_waves / 4;
        if (wgs > cap) wgs = cap;
        const dim3 g{uint32_t(wgs), 1, 1};
        if (rows <= 2) {
            hipLaunchKernelGGL((bigadd_coop_kernel<W, 1, 2, NT>), g, dim3(128), 0, st, a, b, o, carry, uint32_t(m), batch);
        } else if (rows <= 4) {
            hipLaunchKernelGGL((bigadd_coop_kernel<W, 1, 4, NT>), g, dim3(256), 0, st, a, b, o, carry, uint32_t(m), batch);
        } else if (rows <= 8) {
            hipLaunchKernelGGL((bigadd_coop_kernel<W, 2, 4, NT>), g, dim3(256), 0, st, a, b, o, carry, uint32_t(m), batch);
        } else if (rows <= 16) {
            hipLaunchKernelGGL((bigadd_coop_kernel<W, 2, 8, NT>), g, dim3(512), 0, st, a, b, o, carry, uint32_t(m), batch);
        } else {
            hipLaunchKernelGGL((bigadd_coop_kernel<W, 4, 8, NT>), g, dim3(512), 0, st, a, b, o, carry, uint32_t(m), batch);
        }
    }
    return hipGetLastError();
}

template <int W>
static hipError_t launch_w(const uint32_t *a, const uint32_t *b, uint32_t *o, uint8_t *carry, uint64_t m,
                           uint64_t batch, hipStream_t st, const AddTune &t) {
    const uint64_t mw = t.max_waves;
    const bool mu = (m <= 8 * 64) && ((m <= 2 * 64) ? t.multi2 : (m <= 4 * 64) ? t.multi4 : t.multi8);
    if (t.nt) {
        if (t.rows == 2) return launch_wu<W, 2, true>(a, b, o, carry, m, batch, st, mw, mu);
        if (t.rows == 8) return launch_wu<W, 8, true>(a, b, o, carry, m, batch, st, mw, mu);
        return launch_wu<W, 4, true>(a, b, o, carry, m, batch, st, mw, mu);
    }
    if (t.rows == 2) return launch_wu<W, 2, false>(a, b, o, carry, m, batch, st, mw, mu);
    if (t.rows == 8) return launch_wu<W, 8, false>(a, b, o, carry, m, batch, st, mw, mu);
    return launch_wu<W, 4, false>(a, b, o, carry, m, batch, st, mw, mu);
}

hipError_t launch_bigadd_ragged(const void *a, const void *b, void *out, uint8_t *carry, const bi_desc *desc,
                                uint64_t count, uint32_t limb_bits, hipStream_t st, const AddTune &t) {
    if (count == 0) return hipSuccess;
    uint64_t waves = count < t.max_waves ? count : t.max_waves;
    const uint64_t blocks = (waves + 3) / 4;
    auto A = static_cast<const uint32_t *>(a);
    auto B = static_cast<const uint32_t *>(b);
    auto O = static_cast<uint32_t *>(out);
    if (limb_bits == 64)
        hipLaunchKernelGGL((bigadd_ragged_kernel<2, 4>), dim3(uint32_t(blocks)), dim3(256), 0, st, A, B, O, carry, desc, count);
    else
        hipLaunchKernelGGL((bigadd_ragged_kernel<1, 4>), dim3(uint32_t(blocks)), dim3(256), 0, st, A, B, O, carry, desc, count);
    return hipGetLastError();
}

hipError_t launch_bigadd(const void *a, const void *b, void *out, uint8_t *carry, uint64_t inst_bytes,
                         uint64_t batch, hipStream_t st, const AddTune &t) {
    if (batch == 0) return hipSuccess;
    const int cb = pick_chunk_bytes(inst_bytes, a, b, out);
    const uint64_t m = inst_bytes / cb;
    auto A = static_cast<const uint32_t *>(a);
    auto B = static_cast<const uint32_t *>(b);
    auto O = static_cast<uint32_t *>(out);
    switch (cb) {
        case 16: return launch_w<4>(A, B, O, carry, m, batch, st, t);
        case 8: return launch_w<2>(A, B, O, carry, m, batch, st, t);
        default: return launch_w<1>(A, B, O, carry, m, batch, st, t);
    }
}

}  // namespace bi
