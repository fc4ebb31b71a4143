// Fused multi-operation programs (Section 6.1): several same-length
// operations on one instance inside one workgroup, the intermediates kept in
// LDS, the operands read from HBM once and the result written once.
//
//   BI_PROG_ADD6  six additions, a + b, then + a, + b, + a, + b, + a in turn:
//                 4 a + 3 b mod 2^N (the paper names only "six additions";
//                 this alternating chain is the reading taken).
//   BI_PROG_POLY  (a a + b) (b b + b) + a b mod 2^N: four same-length products
//                 (the low n limbs of eq. (1)) and three additions.
//   BI_PROG_MUL_LOW  a b mod 2^N alone: the paper's same-length product of
//                 Figs. 4-5 (only the coefficients below n are formed).
//
// The six additions keep every operand in registers: each lane holds the
// same 4-word chunks of a, b and the running sum throughout.  Instances of up
// to 256 words are packed several to a wave (a segmented ballot-adder: the
// last chunk of an instance neither generates nor propagates into the next),
// larger ones take a workgroup whose waves exchange one carry summary per
// addition.  In Poly every addition is a workgroup ballot-adder pass
// (Section 2) from LDS to LDS.
// A same-length product is the VALU schoolbook of Section 3 restricted to the
// output words below n: waves take blocks of 64 Q consecutive coefficients in
// a snake order (cost grows with the block index), the factor read uniformly
// from LDS is the scalar operand of v_mad_u64_u32 and the other factor is read
// as a sliding window from a zero-padded LDS buffer; each lane folds its Q
// (accumulator, overflow count) pairs into Q low words (written to the result
// buffer) and a (high, carry) pair, and a ballot-adder pass adds the pairs in
// place.  Words at or above n are dropped: arithmetic is mod 2^N.
// Products and Poly of up to 256 words instead run several instances per
// wavefront (fused_packed_kernel): an instance takes a segment of lanes, its
// operands sit in the wavefront's own LDS areas (the per-lane factor is then
// a VGPR operand), the (high, carry) pair moves to the next lane by a lane
// shuffle and the segment's chunks are added with one ballot-adder step, so
// Poly's intermediates stay in registers but for the two factors of its last
// product.
#include <algorithm>
#include <atomic>

#include "bi_common.hpp"
#include "bi_internal.hpp"
#include "bi_valu.hpp"
#include "bi_wgadd.hpp"

namespace bi {

// Longest instance (32-bit words) of the packed product / Poly kernels.
constexpr uint32_t kPackedMaxWords = 256;

namespace {

// Zero words on each side of a buffer used as the windowed factor of a
// product: a block spans 64 Q coefficients and its step loop runs in groups
// of 4, so the window reaches 64 Q + 3 words below 0 and 64 Q words above n.
template <int Q> constexpr uint32_t fused_pad() { return 64 * Q + 4; }

// x = X + Y over n words, in place in LDS.
struct AddSrc {
    const uint32_t *X, *Y;
    uint32_t n;
    __device__ __forceinline__ void operator()(uint32_t c, uint32_t (&x)[4], uint32_t (&y)[4]) const {
        const uint4 u = *reinterpret_cast<const uint4 *>(X + 4 * c);
        const uint4 v = *reinterpret_cast<const uint4 *>(Y + 4 * c);
        x[0] = u.x; x[1] = u.y; x[2] = u.z; x[3] = u.w;
        y[0] = v.x; y[1] = v.y; y[2] = v.z; y[3] = v.w;
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if (4 * c + t >= n) { x[t] = 0; y[t] = 0; }
    }
};

struct LdsSink {
    uint32_t *Z;
    uint32_t n;
    __device__ __forceinline__ void operator()(uint32_t c, const uint32_t (&s)[4]) const {
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if (4 * c + t < n) Z[4 * c + t] = s[t];
    }
};

template <int NW>
__device__ __forceinline__ void wg_add_lds(uint32_t *Z, const uint32_t *X, const uint32_t *Y, uint32_t n,
                                           uint32_t *summary) {
    (void)wg_add_rows_sink<NW>(AddSrc{X, Y, n}, LdsSink{Z, n}, n, summary);
    __syncthreads();
}

// Low n words of the (Q low words, high / carry pair) per lane group: H of
// group g belongs at words Q (g + 1) and Q (g + 1) + 1.
template <int Q>
struct MulLowSrc {
    const uint32_t *L;
    const uint2 *H;
    uint32_t n;
    __device__ __forceinline__ void operator()(uint32_t c, uint32_t (&x)[4], uint32_t (&y)[4]) const {
        const uint4 l = *reinterpret_cast<const uint4 *>(L + 4 * c);
        x[0] = l.x; x[1] = l.y; x[2] = l.z; x[3] = l.w;
        if constexpr (Q == 4) {
            if (c >= 1) {
                const uint2 h = H[c - 1];
                y[0] = h.x; y[1] = h.y;
            }
        } else {
            if (c >= 1) {
                const uint2 h = H[2 * c - 1];
                y[0] = h.x; y[1] = h.y;
            }
            const uint2 h2 = H[2 * c];
            y[2] = h2.x; y[3] = h2.y;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if (4 * c + t >= n) { x[t] = 0; y[t] = 0; }
    }
};

// Z = (U V) mod 2^(32 n).  U: read uniformly, words up to n + 2 (zero above
// n); V: zero at least fused_pad<Q>() words on each side; Z: n words (may not
// alias U or V); H: scratch of 64 entries per block.
template <int Q, int NW>
__device__ __forceinline__ void wg_mul_low(uint32_t *Z, const uint32_t *U, const uint32_t *V, uint2 *H, uint32_t n,
                                           uint32_t *summary) {
    constexpr uint32_t span = 64 * Q;
    const uint32_t lane = lane_id(), wave = wave_in_block();
    const uint32_t NB = (n + span - 1) / span;
    for (uint32_t r = 0;; ++r) {
        const uint32_t slot = (r & 1u) ? (NW - 1 - wave) : wave;  // snake over rising block costs
        const uint32_t blk = r * NW + slot;
        if (blk >= NB) break;
        const uint32_t k0 = blk * span, kl = k0 + Q * lane;
        const uint32_t ihi = min(k0 + span - 1, n - 1);  // steps i <= k for every coefficient k of the block
        uint64_t acc[Q];
        uint32_t cnt[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) { acc[q] = 0; cnt[q] = 0; }
        // window w[q] = V[kl + q - i] at the current step i
        uint32_t w[4];
        auto window = [&](int32_t at, uint32_t (&x)[4]) {
            if constexpr (Q == 4) {
                const uint4 v = *reinterpret_cast<const uint4 *>(V + at);
                x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
            } else {
                const uint2 v0 = *reinterpret_cast<const uint2 *>(V + at);
                const uint2 v1 = *reinterpret_cast<const uint2 *>(V + at + 2);
                x[0] = v0.x; x[1] = v0.y; x[2] = v1.x; x[3] = v1.y;
            }
        };
        window(int32_t(kl), w);
        for (uint32_t i = 0; i <= ihi; i += 4) {
            uint32_t x[4];  // V[kl - i - 4 .. kl - i - 1]
            window(int32_t(kl) - int32_t(i) - 4, x);
            uint32_t av[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) av[u] = __builtin_amdgcn_readfirstlane(U[i + u]);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const int t = q - u + 4;
                    mac(acc[q], cnt[q], av[u], t >= 4 ? w[t - 4] : x[t]);
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) w[q] = x[q];
        }
        // position p collects lo(acc[p]) + hi(acc[p-1]) + cnt[p-2] and the running carry
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
        for (int q = 0; q < Q; ++q)
            if (kl + q < n) Z[kl + q] = R[q];
        H[blk * 64 + lane] = make_uint2(R[Q], R[Q + 1]);
    }
    __syncthreads();
    // Z = L + H in place: each chunk is read and written by the same lane
    (void)wg_add_rows_sink<NW>(MulLowSrc<Q>{Z, H, n}, LdsSink{Z, n}, n, summary);
    __syncthreads();
}

__device__ __forceinline__ void load_operand(uint32_t *dst, const uint32_t *src, uint32_t n) {
    for (uint32_t t = threadIdx.x; t < n; t += blockDim.x) dst[t] = src[t];
}

// A lane's 4-word chunk c of an n-word operand (zero past n or when invalid).
__device__ __forceinline__ void load_chunk(const uint32_t *p, uint32_t n, uint32_t c, bool valid, uint32_t (&x)[4]) {
    const uint32_t base = 4 * c;
    if (valid && base + 4 <= n && (reinterpret_cast<uintptr_t>(p + base) & 15) == 0) {
        const uint4 v = *reinterpret_cast<const uint4 *>(p + base);
        x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
    } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) x[t] = (valid && base + t < n) ? p[base + t] : 0u;
    }
}

// Stores the words of chunk c below n when valid.
__device__ __forceinline__ void store_chunk(uint32_t *p, uint32_t n, uint32_t c, bool valid, const uint32_t (&x)[4]) {
    if (!valid) return;
    const uint32_t base = 4 * c;
    if (base + 4 <= n && (reinterpret_cast<uintptr_t>(p + base) & 15) == 0) {
        *reinterpret_cast<uint4 *>(p + base) = make_uint4(x[0], x[1], x[2], x[3]);
    } else {
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if (base + t < n) p[base + t] = x[t];
    }
}

}  // namespace

// Instances of up to 256 words (64 chunks): 64 / 2^seg_log instances per
// wave, lane j of segment s holding chunk j of instance s.  `keep` masks the
// lanes whose carry may reach the next lane: not an instance's last chunk
// (its carry out is dropped, mod 2^N) and not past the instance's end.
__global__ __launch_bounds__(256) void fused_add6_packed_kernel(const uint32_t *__restrict__ a,
                                                                const uint32_t *__restrict__ b,
                                                                uint32_t *__restrict__ out, uint32_t n,
                                                                uint64_t batch, uint32_t seg_log) {
    const uint32_t lane = lane_id(), wave = wave_in_block();
    const uint32_t nchunks = (n + 3) / 4, ipw = 64u >> seg_log;
    const uint32_t j = lane & ((1u << seg_log) - 1u);
    for (uint64_t g = uint64_t(blockIdx.x) * 4 + wave; g * ipw < batch; g += uint64_t(gridDim.x) * 4) {
        const uint64_t inst = g * ipw + (lane >> seg_log);
        const bool valid = inst < batch && j < nchunks;
        uint32_t A[4], B[4], X[4];
        load_chunk(a + inst * n, n, j, valid, A);
        load_chunk(b + inst * n, n, j, valid, B);
        const uint64_t keep = ballot(valid && j + 1 < nchunks);
        auto add = [&](const uint32_t (&y)[4]) {
            uint32_t s[4];
            const uint32_t gen = add_words<4>(X, y, s);
            const uint64_t G = ballot(gen != 0) & keep, P = ballot(all_ones<4>(s)) & keep;
            add_carry_words<4>(s, uint32_t(wave_carry(G, P, 0).into >> lane) & 1u);
#pragma unroll
            for (int t = 0; t < 4; ++t) X[t] = s[t];
        };
#pragma unroll
        for (int t = 0; t < 4; ++t) X[t] = A[t];
        add(B);
        add(A);
        add(B);
        add(A);
        add(B);
        add(A);
        store_chunk(out + inst * n, n, j, valid, X);
    }
}

// Instances above 256 words: one workgroup of NW waves, wave w holding rows
// w R .. w R + R - 1 (64 chunks each) in registers.  Per addition each wave
// scans its rows, publishes (carry out, all-propagate) in one LDS word,
// and after one barrier applies the carry from the waves below; the summary
// words alternate between two arrays so one barrier per addition suffices.
template <int NW, int R>
__global__ __launch_bounds__(64 * NW) void fused_add6_rows_kernel(const uint32_t *__restrict__ a,
                                                                  const uint32_t *__restrict__ b,
                                                                  uint32_t *__restrict__ out, uint32_t n,
                                                                  uint64_t batch) {
    __shared__ uint32_t summary[2][NW];
    const uint32_t lane = lane_id(), w = wave_in_block();
    const uint32_t nchunks = (n + 3) / 4;
    for (uint64_t q = blockIdx.x; q < batch; q += gridDim.x) {
        uint32_t A[R][4], B[R][4], X[R][4];
        uint64_t vmask[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t row = w * R + r, c = row * 64 + lane;
            const bool valid = c < nchunks;
            load_chunk(a + q * n, n, c, valid, A[r]);
            load_chunk(b + q * n, n, c, valid, B[r]);
            vmask[r] = ballot(valid);
#pragma unroll
            for (int t = 0; t < 4; ++t) X[r][t] = A[r][t];
        }
        uint32_t par = 0;
        auto add = [&](const uint32_t (&y)[R][4]) {
            uint32_t s[R][4];
            uint64_t G[R], P[R];
            uint32_t cin = 0, allp = 1;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint32_t gen = add_words<4>(X[r], y[r], s[r]);
                G[r] = ballot(gen != 0) & vmask[r];
                P[r] = ballot(all_ones<4>(s[r])) & vmask[r];
                cin = wave_carry(G[r], P[r], cin).out;  // past the last chunk: dropped (mod 2^N)
                allp &= P[r] == vmask[r] ? 1u : 0u;
            }
            if (lane == 0) summary[par][w] = cin | (allp << 1);
            __syncthreads();
            cin = 0;
#pragma unroll
            for (int v = 0; v < NW; ++v) {
                const uint32_t sv = summary[par][v];
                if (v < int(w)) cin = (sv & 1u) | ((sv >> 1) & cin);
            }
            par ^= 1u;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const WaveCarry wc = wave_carry(G[r], P[r], cin);
                add_carry_words<4>(s[r], uint32_t(wc.into >> lane) & 1u);
                cin = wc.out;
#pragma unroll
                for (int t = 0; t < 4; ++t) X[r][t] = s[r][t];
            }
        };
        add(B);
        add(A);
        add(B);
        add(A);
        add(B);
        add(A);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t c = (w * R + r) * 64 + lane;
            store_chunk(out + q * n, n, c, c < nchunks, X[r]);
        }
    }
}

// LDS of the polynomial program: four padded buffers (a, b and two
// intermediates at most are live at once) and the products' H scratch.
struct PolyLayout {
    uint32_t stride, pad, h_off, sum_off, words;
};

static PolyLayout poly_layout(uint32_t n, int Q, int NW) {
    PolyLayout l;
    l.pad = 64 * Q + 4;
    l.stride = ((n + 3) & ~3u) + 2 * l.pad;
    const uint32_t NB = (n + 64 * Q - 1) / (64 * Q);
    l.h_off = 4 * l.stride;
    l.sum_off = l.h_off + 2 * NB * 64;
    l.words = l.sum_off + NW;
    return l;
}

template <int Q, int NW>
__global__ __launch_bounds__(64 * NW) void fused_poly_kernel(const uint32_t *__restrict__ a,
                                                             const uint32_t *__restrict__ b, uint32_t *__restrict__ out,
                                                             uint32_t n, uint64_t batch) {
    extern __shared__ __align__(16) uint32_t lds[];
    constexpr uint32_t pad = fused_pad<Q>();
    const uint32_t stride = ((n + 3) & ~3u) + 2 * pad;
    const uint32_t NB = (n + 64 * Q - 1) / (64 * Q);
    uint32_t *buf[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) buf[k] = lds + k * stride + pad;
    uint2 *H = reinterpret_cast<uint2 *>(lds + 4 * stride);
    uint32_t *summary = lds + 4 * stride + 2 * NB * 64;
    // pads and tails are zero for the whole launch: results only write [0, n)
    for (uint32_t t = threadIdx.x; t < 4 * stride; t += 64 * NW) lds[t] = 0;
    __syncthreads();
    for (uint64_t q = blockIdx.x; q < batch; q += gridDim.x) {
        uint32_t *A = buf[0], *B = buf[1], *Z1 = buf[2], *Z2 = buf[3];
        load_operand(A, a + q * n, n);
        load_operand(B, b + q * n, n);
        __syncthreads();
        wg_mul_low<Q, NW>(Z1, A, B, H, n, summary);  // a b
        wg_mul_low<Q, NW>(Z2, A, A, H, n, summary);  // a a
        wg_add_lds<NW>(Z2, Z2, B, n, summary);        // a a + b
        wg_mul_low<Q, NW>(A, B, B, H, n, summary);    // b b (a is no longer needed)
        wg_add_lds<NW>(A, A, B, n, summary);          // b b + b
        wg_mul_low<Q, NW>(B, Z2, A, H, n, summary);   // (a a + b)(b b + b)
        wg_add_rows<NW>(AddSrc{B, Z1, n}, out + q * n, n, summary);
        __syncthreads();
    }
}

// Same-length product alone: a and b in two padded buffers, the result
// formed in a third and copied out.
template <int Q, int NW>
__global__ __launch_bounds__(64 * NW) void fused_mullow_kernel(const uint32_t *__restrict__ a,
                                                               const uint32_t *__restrict__ b,
                                                               uint32_t *__restrict__ out, uint32_t n, uint64_t batch) {
    extern __shared__ __align__(16) uint32_t lds[];
    constexpr uint32_t pad = fused_pad<Q>();
    const uint32_t stride = ((n + 3) & ~3u) + 2 * pad;
    const uint32_t NB = (n + 64 * Q - 1) / (64 * Q);
    uint32_t *U = lds + pad, *V = U + stride, *Z = V + stride;
    uint2 *H = reinterpret_cast<uint2 *>(lds + 3 * stride);
    uint32_t *summary = lds + 3 * stride + 2 * NB * 64;
    for (uint32_t t = threadIdx.x; t < 3 * stride; t += 64 * NW) lds[t] = 0;
    __syncthreads();
    for (uint64_t q = blockIdx.x; q < batch; q += gridDim.x) {
        load_operand(U, a + q * n, n);
        load_operand(V, b + q * n, n);
        __syncthreads();
        wg_mul_low<Q, NW>(Z, U, V, H, n, summary);
        for (uint32_t t = threadIdx.x; t < n; t += 64 * NW) out[q * n + t] = Z[t];
        __syncthreads();
    }
}

namespace {

// ---- Packed small instances (n <= 64 Q words): several per wavefront ----
//
// An instance takes a segment of S = 2^seg_log lanes (S Q >= n); lane j of it
// owns output words Q j .. Q j + Q - 1.  The operands of a product sit in the
// wavefront's own LDS areas, each with at least n + 4 zero words below word 0
// and zeros from word n up to S Q + 4, so the sliding window of the
// multiplicand never needs a bounds check.  Carries between a lane and the
// next one of its segment come from one ballot-adder step (the lanes of an
// instance's last chunk, and lanes past it, neither generate nor propagate).

// Adds y into the lane's Q-word chunk x with carries across the segment.
template <int Q>
__device__ __forceinline__ void seg_add(uint32_t (&x)[Q], const uint32_t (&y)[Q], uint64_t keep, uint32_t lane) {
    uint32_t s[Q];
    const uint32_t g = add_words<Q>(x, y, s);
    const uint64_t G = ballot(g != 0) & keep, P = ballot(all_ones<Q>(s)) & keep;
    add_carry_words<Q>(s, uint32_t(wave_carry(G, P, 0).into >> lane) & 1u);
#pragma unroll
    for (int q = 0; q < Q; ++q) x[q] = s[q];
}

// Four words of V from `at` (16- or two 8-byte LDS reads).
template <int Q>
__device__ __forceinline__ void seg_window(const uint32_t *V, int32_t at, uint32_t (&x)[4]) {
    if constexpr (Q == 4) {
        const uint4 v = *reinterpret_cast<const uint4 *>(V + at);
        x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
    } else {
        const uint2 v0 = *reinterpret_cast<const uint2 *>(V + at);
        const uint2 v1 = *reinterpret_cast<const uint2 *>(V + at + 2);
        x[0] = v0.x; x[1] = v0.y; x[2] = v1.x; x[3] = v1.y;
    }
}

// Z = this lane's chunk of (U V) mod 2^(32 n), U and V the LDS areas of the
// lane's instance.  Each lane accumulates its Q coefficients over every step
// i < n (steps above a coefficient read the zeros below V), folds them into
// Q low words and a (high, carry) pair that belongs to the next lane's first
// two words, and the chunks are then added across the segment.
template <int Q>
__device__ __forceinline__ void seg_mul_low(const uint32_t *U, const uint32_t *V, uint32_t n, uint32_t j,
                                            uint64_t keep, uint32_t lane, uint32_t (&Z)[Q]) {
    const uint32_t kl = Q * j;
    uint64_t acc[Q];
    uint32_t cnt[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) { acc[q] = 0; cnt[q] = 0; }
    uint32_t w[4];  // V[kl .. kl + 3]
    seg_window<Q>(V, int32_t(kl), w);
    for (uint32_t i = 0; i < n; i += 4) {
        uint32_t x[4];  // V[kl - i - 4 .. kl - i - 1]
        seg_window<Q>(V, int32_t(kl) - int32_t(i) - 4, x);
        const uint4 a4 = *reinterpret_cast<const uint4 *>(U + i);
        const uint32_t av[4] = {a4.x, a4.y, a4.z, a4.w};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int t = q - u + 4;
                mac_v(acc[q], cnt[q], av[u], t >= 4 ? w[t - 4] : x[t]);
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) w[q] = x[q];
    }
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
    uint32_t h0 = __shfl_up(R[Q], 1), h1 = __shfl_up(R[Q + 1], 1);
    if (j == 0) { h0 = 0; h1 = 0; }
    uint32_t y[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) { Z[q] = R[q]; y[q] = q == 0 ? h0 : q == 1 ? h1 : 0u; }
    seg_add<Q>(Z, y, keep, lane);
}

// Words Q j .. Q j + Q - 1 of an n-word operand (zero past n or when invalid).
template <int Q>
__device__ __forceinline__ void load_q(const uint32_t *p, uint32_t n, uint32_t j, bool valid, uint32_t (&x)[Q]) {
#pragma unroll
    for (int q = 0; q < Q; ++q) x[q] = (valid && Q * j + q < n) ? p[Q * j + q] : 0u;
}

template <int Q>
__device__ __forceinline__ void store_q(uint32_t *p, uint32_t n, uint32_t j, bool valid, const uint32_t (&x)[Q]) {
    if (!valid) return;
#pragma unroll
    for (int q = 0; q < Q; ++q)
        if (Q * j + q < n) p[Q * j + q] = x[q];
}

// Words per LDS operand area: the zeros below (>= n + 4, a multiple of 4)
// and S Q + 4 words from word 0, rounded to a multiple of 4.
__host__ __device__ inline uint32_t packed_pad(uint32_t n) { return (n + 7) & ~3u; }
__host__ __device__ inline uint32_t packed_area(uint32_t n, uint32_t sq) { return packed_pad(n) + ((sq + 7) & ~3u); }

}  // namespace

// Same-length product (PROG = BI_PROG_MUL_LOW) or Poly (BI_PROG_POLY) of
// instances of at most 64 Q words, 64 / 2^seg_log per wavefront, one
// wavefront per workgroup.  LDS: per instance 2 (product) or 4 (Poly)
// operand areas.  Poly keeps a b in registers, forms a a + b and b b + b in
// registers and stores them as the operands of the last product.
template <int Q, int PROG>
__global__ __launch_bounds__(64) void fused_packed_kernel(const uint32_t *__restrict__ a,
                                                          const uint32_t *__restrict__ b, uint32_t *__restrict__ out,
                                                          uint32_t n, uint64_t batch, uint32_t seg_log) {
    extern __shared__ __align__(16) uint32_t lds[];
    constexpr uint32_t NA = PROG == BI_PROG_POLY ? 4 : 2;
    const uint32_t lane = lane_id(), S = 1u << seg_log, ipw = 64u >> seg_log;
    const uint32_t j = lane & (S - 1u), slot = lane >> seg_log;
    const uint32_t nq = (n + Q - 1) / Q;  // chunks per instance
    const uint32_t aw = packed_area(n, S * Q);
    for (uint32_t t = lane; t < ipw * NA * aw; t += 64) lds[t] = 0;
    __syncthreads();
    uint32_t *area[NA];
#pragma unroll
    for (uint32_t k = 0; k < NA; ++k) area[k] = lds + (slot * NA + k) * aw + packed_pad(n);
    for (uint64_t g = blockIdx.x; g * ipw < batch; g += gridDim.x) {
        const uint64_t inst = g * ipw + slot;
        const bool valid = inst < batch && j < nq;
        const uint64_t keep = ballot(valid && j + 1 < nq);
        uint32_t A[Q], Bv[Q], Z[Q];
        load_q<Q>(a + inst * n, n, j, valid, A);
        load_q<Q>(b + inst * n, n, j, valid, Bv);
        store_q<Q>(area[0], n, j, valid, A);
        store_q<Q>(area[1], n, j, valid, Bv);
        __syncthreads();
        seg_mul_low<Q>(area[0], area[1], n, j, keep, lane, Z);  // a b
        if constexpr (PROG == BI_PROG_POLY) {
            uint32_t T[Q], U2[Q], R[Q];
            seg_mul_low<Q>(area[0], area[0], n, j, keep, lane, T);  // a a
            seg_add<Q>(T, Bv, keep, lane);                          // a a + b
            seg_mul_low<Q>(area[1], area[1], n, j, keep, lane, U2);  // b b
            seg_add<Q>(U2, Bv, keep, lane);                          // b b + b
            store_q<Q>(area[2], n, j, valid, T);
            store_q<Q>(area[3], n, j, valid, U2);
            __syncthreads();
            seg_mul_low<Q>(area[2], area[3], n, j, keep, lane, R);  // (a a + b)(b b + b)
            seg_add<Q>(R, Z, keep, lane);                           // + a b
#pragma unroll
            for (int q = 0; q < Q; ++q) Z[q] = R[q];
        }
        store_q<Q>(out + inst * n, n, j, valid, Z);
        __syncthreads();  // the areas are rewritten by the next group
    }
}

namespace {

// Packed path parameters for n words: (Q, seg_log), Q = 0 when n is too long.
struct PackedPlan {
    int Q = 0;
    uint32_t seg_log = 0;
};
PackedPlan packed_plan(uint32_t n) {
    PackedPlan p;
    if (n == 0 || n > kPackedMaxWords) return p;
    p.Q = n <= 64 ? 2 : 4;  // 2 measured faster at 32 words (Poly 1.58 vs 1.87 ms), 4 at 128
    const uint32_t lanes = (n + p.Q - 1) / p.Q;
    while ((1u << p.seg_log) < lanes) ++p.seg_log;
    return p;
}
size_t packed_lds_bytes(int program, uint32_t n, const PackedPlan &p) {
    const uint32_t S = 1u << p.seg_log;
    return 4ull * (64u >> p.seg_log) * (program == BI_PROG_POLY ? 4 : 2) * packed_area(n, S * uint32_t(p.Q));
}

// Waves per workgroup for n words: enough 64-chunk rows (six additions) or
// block pairs (products) to give each wave work, a power of two up to 16.
uint32_t pow2_waves(uint32_t units) {
    return units >= 16 ? 16 : units >= 8 ? 8 : units >= 4 ? 4 : units >= 2 ? 2 : 1;
}

// Persistent grid of resident workgroups (each loops over instances).  One
// instantiation per kernel, so each keeps its own occupancy record.
using FusedKernel = void (*)(const uint32_t *, const uint32_t *, uint32_t *, uint32_t, uint64_t);
template <FusedKernel kernel>
hipError_t launch_persistent(uint32_t threads, size_t lds, const uint32_t *a, const uint32_t *b, uint32_t *c,
                             uint32_t n, uint64_t batch, hipStream_t st, int num_cus) {
    const void *fn = reinterpret_cast<const void *>(kernel);
    // ((LDS bytes + 1) << 32 | resident workgroups per CU) of the last launch
    // of this kernel (0: none yet)
    static std::atomic<uint64_t> occ{0}, lds_set{0};
    hipError_t e = hipSuccess;
    if (lds > 0) {  // kernels with dynamic LDS may use all of a CU's
        e = lds_limit_once(fn, lds_set);
        if (e != hipSuccess) return e;
    }
    uint64_t o = occ.load(std::memory_order_relaxed);
    if ((o >> 32) != lds + 1) {
        int nblk = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nblk, fn, int(threads), lds);
        if (e != hipSuccess) return e;
        o = (uint64_t(lds + 1) << 32) | uint32_t(nblk < 1 ? 1 : nblk);
        occ.store(o, std::memory_order_relaxed);
    }
    const uint64_t cap = uint64_t(uint32_t(o)) * uint64_t(num_cus > 0 ? num_cus : 1);
    const uint32_t grid = uint32_t(batch < cap ? batch : cap);
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(threads), lds, st, a, b, c, n, batch);
    return hipGetLastError();
}

}  // namespace

// LDS words of the same-length product: three padded buffers, H, summary.
static uint32_t mullow_lds_words(uint32_t n, int Q, int NW) {
    const uint32_t stride = ((n + 3) & ~3u) + 2 * (64 * Q + 4);
    const uint32_t NB = (n + 64 * Q - 1) / (64 * Q);
    return 3 * stride + 2 * NB * 64 + NW;
}

size_t fused_lds_bytes(int program, uint32_t n32) {
    if (program == BI_PROG_ADD6) return 0;  // registers only
    const PackedPlan pp = packed_plan(n32);
    if (pp.Q != 0) return packed_lds_bytes(program, n32, pp);
    const int Q = n32 > 4096 ? 4 : 2;
    const uint32_t NB = (n32 + 64 * Q - 1) / (64 * Q);
    const int nw = int(pow2_waves((NB + 1) / 2));
    if (program == BI_PROG_MUL_LOW) return 4ull * mullow_lds_words(n32, Q, nw);
    return 4ull * poly_layout(n32, Q, nw).words;
}

hipError_t launch_fused(int program, const uint32_t *a, const uint32_t *b, uint32_t *c, uint32_t n, uint64_t batch,
                        hipStream_t st, int num_cus) {
    if (batch == 0) return hipSuccess;
    if (program == BI_PROG_ADD6) {
        const uint32_t nchunks = (n + 3) / 4, rows = (nchunks + 63) / 64;
        if (rows == 1) {
            uint32_t seg_log = 0;
            while ((1u << seg_log) < nchunks) ++seg_log;
            const uint64_t waves = (batch + (64u >> seg_log) - 1) / (64u >> seg_log);
            const uint64_t cap = uint64_t(num_cus > 0 ? num_cus : 1) * 32;
            const uint32_t grid = uint32_t(std::min((waves + 3) / 4, cap));
            hipLaunchKernelGGL(fused_add6_packed_kernel, dim3(grid), dim3(256), 0, st, a, b, c, n, batch, seg_log);
            return hipGetLastError();
        }
        // up to 4 rows per lane group: fewer waves per instance, more
        // instances resident per CU to hide the per-addition barrier
        uint32_t nw = 1;
        while (4 * nw < rows) nw *= 2;
        const uint32_t r = (rows + nw - 1) / nw;
#define BI_ADD6_CASE(W, RR) \
    if (nw == W && r == RR) return launch_persistent<&fused_add6_rows_kernel<W, RR>>(64 * W, 0, a, b, c, n, batch, st, num_cus);
        BI_ADD6_CASE(1, 2) BI_ADD6_CASE(1, 3) BI_ADD6_CASE(1, 4) BI_ADD6_CASE(2, 3) BI_ADD6_CASE(2, 4)
        BI_ADD6_CASE(4, 3) BI_ADD6_CASE(4, 4) BI_ADD6_CASE(8, 3) BI_ADD6_CASE(8, 4)
#undef BI_ADD6_CASE
        return hipErrorInvalidValue;
    }
    const PackedPlan pp = packed_plan(n);
    if (pp.Q != 0) {
        const size_t lds = packed_lds_bytes(program, n, pp);
        const uint64_t waves = (batch + (64u >> pp.seg_log) - 1) / (64u >> pp.seg_log);
        const uint32_t grid = uint32_t(std::min<uint64_t>(waves, uint64_t(num_cus > 0 ? num_cus : 1) * 32));
#define BI_PACKED_CASE(QQ, PR)                                                                                      \
    if (pp.Q == QQ && program == PR) {                                                                              \
        hipLaunchKernelGGL((fused_packed_kernel<QQ, PR>), dim3(grid), dim3(64), lds, st, a, b, c, n, batch,         \
                           pp.seg_log);                                                                             \
        return hipGetLastError();                                                                                   \
    }
        BI_PACKED_CASE(2, BI_PROG_MUL_LOW) BI_PACKED_CASE(4, BI_PROG_MUL_LOW)
        BI_PACKED_CASE(2, BI_PROG_POLY) BI_PACKED_CASE(4, BI_PROG_POLY)
#undef BI_PACKED_CASE
        return hipErrorInvalidValue;
    }
    const int Q = n > 4096 ? 4 : 2;
    const uint32_t NB = (n + 64 * Q - 1) / (64 * Q);
    const uint32_t nw = pow2_waves((NB + 1) / 2);
    if (program == BI_PROG_MUL_LOW) {
        const size_t lds = 4ull * mullow_lds_words(n, Q, int(nw));
#define BI_MULLOW_CASE(QQ, W)                                                                                       \
    if (Q == QQ && nw == W)                                                                                         \
        return launch_persistent<&fused_mullow_kernel<QQ, W>>(64 * W, lds, a, b, c, n, batch, st, num_cus);
        BI_MULLOW_CASE(2, 1) BI_MULLOW_CASE(2, 2) BI_MULLOW_CASE(2, 4) BI_MULLOW_CASE(2, 8) BI_MULLOW_CASE(2, 16)
        BI_MULLOW_CASE(4, 1) BI_MULLOW_CASE(4, 2) BI_MULLOW_CASE(4, 4) BI_MULLOW_CASE(4, 8) BI_MULLOW_CASE(4, 16)
#undef BI_MULLOW_CASE
        return hipErrorInvalidValue;
    }
    const size_t lds = 4ull * poly_layout(n, Q, int(nw)).words;
#define BI_POLY_CASE(QQ, W)                                                                                         \
    if (Q == QQ && nw == W)                                                                                         \
        return launch_persistent<&fused_poly_kernel<QQ, W>>(64 * W, lds, a, b, c, n, batch, st, num_cus);
    BI_POLY_CASE(2, 1) BI_POLY_CASE(2, 2) BI_POLY_CASE(2, 4) BI_POLY_CASE(2, 8) BI_POLY_CASE(2, 16)
    BI_POLY_CASE(4, 1) BI_POLY_CASE(4, 2) BI_POLY_CASE(4, 4) BI_POLY_CASE(4, 8) BI_POLY_CASE(4, 16)
#undef BI_POLY_CASE
    return hipErrorInvalidValue;
}

}  // namespace bi
