// Addition of one integer too long for one workgroup (Section 2's addition
// as a carry scan, carried across workgroups; the paper leaves such sizes to
// its slower fall-back versions, Section 5.1).
//
// Four stream-ordered kernels (the fix-up is two); no workgroup ever waits
// on another:
//  1. tile pass: the integer is cut into tiles of NW waves x U rows x 64
//     chunks of W words.  A tile is added with carry-in 0 through the same
//     thread -> wave -> workgroup ballot-adder hierarchy as the cooperative
//     batched schedule, its sum is stored, and it is reduced to a summary:
//     g (the tile carries out with carry-in 0) and p (the tile's sum is all
//     ones, so a carry-in passes through it); never both.
//  2. summary scan: one workgroup scans the summaries with the carry
//     operator (g1, p1) then (g2, p2) -> (g2 | p2 & g1, p1 & p2) into each
//     tile's true carry-in and the carry out of the integer.
//  3. fix-up: a tile whose carry-in is 1 adds it into its stored sum; the
//     words up to and including the first one that is not all ones change
//     (all-ones words wrap to 0, that word increments).  A lane per tile
//     handles the usual case, where the tile's first chunk is not all ones,
//     and appends the other tiles to a list; a second kernel walks each
//     listed tile with a wavefront, a row of 64 chunks per step (carries
//     through long all-ones runs then still spread over the whole GPU).
// HBM traffic is one pass (read a and b, write the sum) plus the summaries and
// the fix-up's few chunks.  A single-pass decoupled look-back scan would save
// the summary round trip but makes workgroups spin on their predecessors.
//
// Up to 512 tiles (2^21 words in 16-byte chunks) two kernels do instead,
// where the four launches' latency outweighs a second read of a and b: a
// summary pass, then a pass that finds each tile's carry-in from the
// summaries below it (the nearest tile that does not only propagate gives
// its own carry out) and stores the final sum.  Measured on one 2^20 /
// 2^24 / 2^28-bit pair: 14.0 / 13.7 / 28.0 -> 11.7 / 11.4 / 32.9 us with two
// passes (all-ones plus one: 19.9 / 21.8 / 48.5 -> 12.0 / 11.4 / 35.4 us).
//
// The chunk width W (16, 8 or 4 bytes) follows the pointers' alignment; the
// integer's length need not be a multiple of it: the missing words of the
// last chunk read as all ones in a and zero in b (and as all ones when the
// fix-up reads the sum), which passes carries through unchanged, and are
// never stored.
#include <algorithm>

#include "bi_common.hpp"
#include "bi_internal.hpp"

namespace bi {

namespace {

constexpr int kLargeNW = 4;  // waves per tile-pass workgroup
constexpr int kLargeU = 4;   // rows of 64 chunks per wave
constexpr int kRowsPerTile = kLargeNW * kLargeU;
constexpr int kScanThreads = 1024;
constexpr uint64_t kMaxTileGrid = uint64_t(1) << 22;  // workgroups of the tile pass
constexpr uint64_t kTwoPassTiles = 512;                // up to this many tiles: two passes

// Summary bytes are padded to whole 16-byte words; padding is never read as
// a tile.
__host__ __device__ inline uint64_t summary_stride(uint64_t tiles) { return (tiles + 15) & ~uint64_t(15); }

// Chunk c of a W-word chunked array of n32 words (m chunks, the last one
// holding `tail` words); missing words read as `pad`.
template <int W, bool NT>
__device__ __forceinline__ void load_chunk(const uint32_t *p, uint64_t c, uint64_t m, uint32_t tail, uint32_t pad,
                                           uint32_t (&v)[W]) {
    if (c + 1 < m || tail == W) {
        load_words<W, NT>(p + c * W, v);
    } else {
#pragma unroll
        for (int w = 0; w < W; ++w) v[w] = uint32_t(w) < tail ? p[c * W + w] : pad;
    }
}

template <int W, bool NT>
__device__ __forceinline__ void store_chunk(uint32_t *p, uint64_t c, uint64_t m, uint32_t tail, const uint32_t (&v)[W]) {
    if (c + 1 < m || tail == W) {
        store_words<W, NT>(p + c * W, v);
    } else {
#pragma unroll
        for (int w = 0; w < W; ++w)
            if (uint32_t(w) < tail) p[c * W + w] = v[w];
    }
}

// MODE kTileSums: store each tile's sum with carry-in 0 and its summary;
// kTileSummary: the summary only; kTileFinal (after a kTileSummary pass):
// take the tile's carry-in from the summaries below it, store the final sum
// and, at the last tile, the carry out of the integer.
enum TileMode { kTileSums, kTileSummary, kTileFinal };

template <int W, bool NT, int MODE = kTileSums>
__global__ __launch_bounds__(64 * kLargeNW) void large_add_tile_kernel(const uint32_t *a, const uint32_t *b,
                                                                       uint32_t *out, uint8_t *summary, uint64_t m,
                                                                       uint32_t tail, uint64_t tiles,
                                                                       uint8_t *carry_out = nullptr) {
    __shared__ uint32_t summ[kLargeNW];
    __shared__ uint32_t tile_cin;
    const uint32_t lane = lane_id();
    const uint32_t wave = wave_in_block();
    const uint64_t rows = (m + 63) / 64;
    for (uint64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        const uint64_t r0 = (t * kLargeNW + wave) * kLargeU;
        uint32_t s[kLargeU][W];
        uint64_t G[kLargeU], P[kLargeU];
#pragma unroll
        for (int u = 0; u < kLargeU; ++u) {
            const uint64_t c = (r0 + u) * 64 + lane;
            uint32_t va[W], vb[W];
#pragma unroll
            for (int w = 0; w < W; ++w) { va[w] = 0; vb[w] = 0; }
            if (c < m) {
                load_chunk<W, NT>(a, c, m, tail, 0xFFFFFFFFu, va);
                load_chunk<W, NT>(b, c, m, tail, 0u, vb);
            }
            const uint32_t g = add_words<W>(va, vb, s[u]);
            G[u] = ballot(g != 0);
            P[u] = ballot(c < m && all_ones<W>(s[u]));
        }
        // Summary of this wave's rows; rows past the end are the identity.
        uint32_t cout = 0, allp = 1;
#pragma unroll
        for (int u = 0; u < kLargeU; ++u) {
            if (r0 + u < rows) {  // uniform
                const uint64_t valid = std::min<uint64_t>(m - (r0 + u) * 64, 64);
                const uint64_t vmask = valid >= 64 ? ~0ull : ((1ull << valid) - 1);
                const WaveCarry wc = wave_carry(G[u], P[u], cout);
                cout = valid >= 64 ? wc.out : uint32_t(wc.into >> valid) & 1u;
                allp &= (P[u] == vmask) ? 1u : 0u;
            }
        }
        if constexpr (MODE == kTileFinal) {
            // the nearest tile below that does not only propagate gives the
            // carry-in (its own carry out); below tile 0 nothing carries.
            // Lanes read tiles t - 1 - lane - 64 q, nearest first.
            if (wave == 0) {
                uint32_t c0 = 0;
                for (int64_t base = int64_t(t) - 1; base >= 0; base -= 64) {
                    const int64_t j = base - int64_t(lane);
                    const uint32_t sv = j >= 0 ? summary[j] : 0u;
                    const uint64_t stop = ballot((sv & 2u) == 0);
                    if (stop) {  // uniform
                        c0 = __shfl(sv, int(__ffsll(static_cast<unsigned long long>(stop)) - 1)) & 1u;
                        break;
                    }
                }
                if (lane == 0) tile_cin = c0;
            }
        }
        if (lane == 0) summ[wave] = cout | (allp << 1);
        __syncthreads();
        const uint32_t tcin = MODE == kTileFinal ? tile_cin : 0u;
        uint32_t cin = tcin, tg = 0, tp = 1;
#pragma unroll
        for (int v = 0; v < kLargeNW; ++v) {
            const uint32_t sv = summ[v];
            if (v < int(wave)) cin = (sv & 1u) | ((sv >> 1) & cin);
            tg = (sv & 1u) | ((sv >> 1) & tg);
            tp &= sv >> 1;
        }
        if constexpr (MODE != kTileSummary) {
#pragma unroll
            for (int u = 0; u < kLargeU; ++u) {
                if (r0 + u < rows) {  // uniform
                    const uint64_t c = (r0 + u) * 64 + lane;
                    const uint64_t valid = std::min<uint64_t>(m - (r0 + u) * 64, 64);
                    const WaveCarry wc = wave_carry(G[u], P[u], cin);
                    add_carry_words<W>(s[u], uint32_t(wc.into >> lane) & 1u);
                    if (c < m) store_chunk<W, NT>(out, c, m, tail, s[u]);
                    cin = valid >= 64 ? wc.out : uint32_t(wc.into >> valid) & 1u;
                }
            }
        }
        if constexpr (MODE == kTileFinal) {
            if (carry_out && t == tiles - 1 && threadIdx.x == 0) *carry_out = uint8_t(tg | (tp & tcin));
        } else {
            if (threadIdx.x == 0) summary[t] = uint8_t(tg | (tp << 1));
        }
        __syncthreads();  // summ and tile_cin are rewritten by the next tile
    }
}

// Folds the summaries in one 16-byte word (tiles t0 .. t0 + 15; bytes at or
// past `tiles` are skipped) into (g, p).
__device__ __forceinline__ void fold_word(const uint4 v, uint64_t t0, uint64_t tiles, uint32_t &g, uint32_t &p) {
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        if (t0 + j < tiles) {
            const uint32_t sv = (w[j >> 2] >> (8 * (j & 3))) & 0xFFu;
            g = (sv & 1u) | ((sv >> 1) & g);
            p &= sv >> 1;
        }
    }
}

// One workgroup: each thread folds a contiguous run of summaries (a whole
// number of 16-byte words, loaded four at a time), the runs are combined by a
// wave-level ballot adder and an LDS pass over the waves, and each thread
// then walks its run again writing every tile's carry-in, a word at a time.
__global__ __launch_bounds__(kScanThreads) void large_add_scan_kernel(const uint4 *summary, uint4 *tile_cin,
                                                                      uint8_t *carry_out, uint32_t *walk_count,
                                                                      uint64_t tiles) {
    __shared__ uint32_t ws[kScanThreads / 64];
    const uint32_t lane = lane_id();
    const uint32_t wave = wave_in_block();
    const uint64_t words = summary_stride(tiles) / 16;
    const uint64_t per = (words + kScanThreads - 1) / kScanThreads;  // words per thread
    const uint64_t w0 = std::min<uint64_t>(uint64_t(threadIdx.x) * per, words);
    const uint64_t w1 = std::min<uint64_t>(w0 + per, words);
    uint32_t g = 0, p = 1;
    uint64_t w = w0;
    for (; w + 4 <= w1; w += 4) {
        uint4 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = summary[w + k];
#pragma unroll
        for (int k = 0; k < 4; ++k) fold_word(v[k], 16 * (w + k), tiles, g, p);
    }
    for (; w < w1; ++w) fold_word(summary[w], 16 * w, tiles, g, p);
    const uint64_t G = ballot(g != 0), P = ballot(p != 0);
    const WaveCarry wz = wave_carry(G, P, 0u);
    if (lane == 0) ws[wave] = wz.out | ((P == ~0ull ? 1u : 0u) << 1);
    __syncthreads();
    uint32_t wcin = 0;
    for (uint32_t v = 0; v < wave; ++v) {
        const uint32_t sv = ws[v];
        wcin = (sv & 1u) | ((sv >> 1) & wcin);
    }
    const WaveCarry wc = wave_carry(G, P, wcin);
    uint32_t c = uint32_t(wc.into >> lane) & 1u;
    if (threadIdx.x == 0) *walk_count = 0;  // read by the fix-up kernels that follow
    for (w = w0; w < w1; ++w) {
        const uint4 v = summary[w];
        const uint32_t in[4] = {v.x, v.y, v.z, v.w};
        uint32_t o[4] = {0, 0, 0, 0};
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            o[j >> 2] |= c << (8 * (j & 3));
            const uint32_t sv = (in[j >> 2] >> (8 * (j & 3))) & 0xFFu;
            if (16 * w + j < tiles) c = (sv & 1u) | ((sv >> 1) & c);
        }
        tile_cin[w] = make_uint4(o[0], o[1], o[2], o[3]);
    }
    if (carry_out && w0 < w1 && w1 == words) *carry_out = uint8_t(c);
}

// Lane l of a wavefront takes tile tb + l.  If the tile's carry-in is 1 and
// its first chunk is not all ones, the carry stops inside that chunk;
// otherwise the tile goes on the walk list (one atomic per wavefront).
template <int W>
__global__ __launch_bounds__(256) void large_add_fixup_kernel(uint32_t *out, const uint8_t *tile_cin, uint64_t m,
                                                              uint32_t tail, uint64_t tiles, uint32_t *walk_list,
                                                              uint32_t *walk_count) {
    const uint32_t lane = lane_id();
    const uint64_t nwaves = (uint64_t(gridDim.x) * blockDim.x) >> 6;
    for (uint64_t tb = wave_global() * 64; tb < tiles; tb += nwaves * 64) {
        const uint64_t tl = tb + lane;
        bool rest = false;
        if (tl < tiles && tile_cin[tl]) {
            const uint64_t c = tl * kRowsPerTile * 64;
            uint32_t s[W];
            load_chunk<W, false>(out, c, m, tail, 0xFFFFFFFFu, s);
            if (all_ones<W>(s)) {
                rest = true;
            } else {
                add_carry_words<W>(s, 1u);
                store_chunk<W, false>(out, c, m, tail, s);
            }
        }
        const uint64_t mask = ballot(rest);
        if (mask) {  // uniform
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(walk_count, uint32_t(__builtin_popcountll(mask)));
            base = __builtin_amdgcn_readfirstlane(base);
            if (rest) walk_list[base + __builtin_popcountll(mask & ((1ull << lane) - 1))] = uint32_t(tl);
        }
    }
}

// One wavefront per listed tile: adds the carry from the tile's first chunk,
// a row of 64 chunks per step, until a chunk that is not all ones.
template <int W>
__global__ __launch_bounds__(256) void large_add_walk_kernel(uint32_t *out, uint64_t m, uint32_t tail,
                                                             const uint32_t *walk_list, const uint32_t *walk_count) {
    const uint32_t lane = lane_id();
    const uint64_t nwaves = (uint64_t(gridDim.x) * blockDim.x) >> 6;
    const uint32_t count = __builtin_amdgcn_readfirstlane(*walk_count);
    for (uint64_t i = wave_global(); i < count; i += nwaves) {
        const uint64_t t = __builtin_amdgcn_readfirstlane(walk_list[i]);
        for (uint32_t r = 0; r < uint32_t(kRowsPerTile); ++r) {
            const uint64_t c = (t * kRowsPerTile + r) * 64 + lane;
            const bool ok = c < m;
            uint32_t s[W];
#pragma unroll
            for (int w = 0; w < W; ++w) s[w] = 0;
            if (ok) load_chunk<W, false>(out, c, m, tail, 0xFFFFFFFFu, s);
            const uint64_t stop = ballot(!ok || !all_ones<W>(s));
            const uint32_t first = stop ? uint32_t(__builtin_ctzll(stop)) : 64u;
            if (ok && lane <= first) {
                add_carry_words<W>(s, 1u);
                store_chunk<W, false>(out, c, m, tail, s);
            }
            if (stop) break;  // uniform
        }
    }
}

template <int W, bool NT>
hipError_t launch_large_w(const uint32_t *a, const uint32_t *b, uint32_t *out, uint8_t *carry, uint64_t n32,
                          uint8_t *scratch, hipStream_t st, int num_cus) {
    const uint64_t m = (n32 + W - 1) / W;
    const uint32_t tail = uint32_t(n32 - (m - 1) * W);
    const uint64_t tiles = large_add_tiles(n32, W);
    const uint64_t stride = summary_stride(tiles);
    uint8_t *summary = scratch;
    uint8_t *tile_cin = scratch + stride;
    uint32_t *walk_list = reinterpret_cast<uint32_t *>(scratch + 2 * stride);
    uint32_t *walk_count = walk_list + stride;
    // One tile per workgroup (the hardware keeps the CUs fed; a persistent
    // grid looping over tiles measured 17 % slower), looping only past 2^22.
    const uint64_t grid = std::min<uint64_t>(tiles, kMaxTileGrid);
    if (tiles <= kTwoPassTiles) {
        // summaries, then every tile's final sum with its carry-in found
        // from them: two launches instead of four; a and b are read twice
        // (the second time mostly from the caches)
        hipLaunchKernelGGL((large_add_tile_kernel<W, false, kTileSummary>), dim3(uint32_t(grid)), dim3(64 * kLargeNW), 0,
                           st, a, b, out, summary, m, tail, tiles, nullptr);
        hipLaunchKernelGGL((large_add_tile_kernel<W, NT, kTileFinal>), dim3(uint32_t(grid)), dim3(64 * kLargeNW), 0, st,
                           a, b, out, summary, m, tail, tiles, carry);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((large_add_tile_kernel<W, NT>), dim3(uint32_t(grid)), dim3(64 * kLargeNW), 0, st, a, b, out,
                       summary, m, tail, tiles, nullptr);
    hipLaunchKernelGGL(large_add_scan_kernel, dim3(1), dim3(kScanThreads), 0, st,
                       reinterpret_cast<const uint4 *>(summary), reinterpret_cast<uint4 *>(tile_cin), carry, walk_count,
                       tiles);
    const uint64_t waves = std::min<uint64_t>((tiles + 63) / 64, uint64_t(num_cus) * 32);
    hipLaunchKernelGGL((large_add_fixup_kernel<W>), dim3(uint32_t((waves + 3) / 4)), dim3(256), 0, st, out, tile_cin,
                       m, tail, tiles, walk_list, walk_count);
    // The list length is known only on the device: a fixed grid of waves
    // reads it and strides over the list.
    const uint64_t walkers = std::min<uint64_t>(tiles, uint64_t(num_cus) * 32);
    hipLaunchKernelGGL((large_add_walk_kernel<W>), dim3(uint32_t((walkers + 3) / 4)), dim3(256), 0, st, out, m, tail,
                       walk_list, walk_count);
    return hipGetLastError();
}

}  // namespace

int large_add_chunk_words(const void *a, const void *b, const void *out) {
    const uintptr_t al = reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b) |
                         reinterpret_cast<uintptr_t>(out);
    return (al & 15) == 0 ? 4 : (al & 7) == 0 ? 2 : 1;
}

// Summaries and carry-ins (a padded byte each), the walk list (a 32-bit
// tile index each) and its length.
size_t large_add_scratch_bytes(uint64_t tiles) { return size_t(6 * summary_stride(tiles) + 16); }

uint64_t large_add_tiles(uint64_t n32, int w) {
    const uint64_t chunks = (n32 + w - 1) / w;
    return (chunks + 64 * kRowsPerTile - 1) / (64 * kRowsPerTile);
}

hipError_t launch_bigadd_large(const void *a, const void *b, void *out, uint8_t *carry, uint64_t n32,
                               uint8_t *scratch, hipStream_t st, int num_cus) {
    auto A = static_cast<const uint32_t *>(a);
    auto B = static_cast<const uint32_t *>(b);
    auto O = static_cast<uint32_t *>(out);
    // Streamed (non-temporal) accesses once the three operands exceed what
    // the caches could keep anyway.
    const bool nt = n32 * 12 > (uint64_t(64) << 20);
    switch (large_add_chunk_words(a, b, out)) {
        case 4: return nt ? launch_large_w<4, true>(A, B, O, carry, n32, scratch, st, num_cus)
                          : launch_large_w<4, false>(A, B, O, carry, n32, scratch, st, num_cus);
        case 2: return nt ? launch_large_w<2, true>(A, B, O, carry, n32, scratch, st, num_cus)
                          : launch_large_w<2, false>(A, B, O, carry, n32, scratch, st, num_cus);
        default: return nt ? launch_large_w<1, true>(A, B, O, carry, n32, scratch, st, num_cus)
                           : launch_large_w<1, false>(A, B, O, carry, n32, scratch, st, num_cus);
    }
}

}  // namespace bi
