// Karatsuba multiplication over the batched products.  The paper picks
// between its schoolbook and FFT kernels by size and leaves sub-quadratic
// splits unexplored (Section 1); here levels of the subtractive Karatsuba
// method reduce a batch of long products to a larger batch of shorter ones
// that the schoolbook (or NTT) kernels run at their most efficient size.
//
// One level turns a product of n-word operands into three products of h
// words, h = ceil(n / 2) rounded up to a multiple of 4: with X = 2^(32 h),
// a = a0 + a1 X and b = b0 + b1 X (a1, b1 zero-padded to h words),
//     z0 = a0 b0,   z2 = a1 b1,   D = |a0 - a1| |b0 - b1|,
//     a b = z0 + X^2 z2 + X (z0 + z2 - s D),
// s = +1 when a0 - a1 and b0 - b1 have the same sign, -1 otherwise (the
// middle term a0 b1 + a1 b0 is never negative).  Levels repeat the split on
// all three products until the operands have at most `base` words; the
// 3^levels products of the last level form one batch for the base algorithm,
// so a pair costs 3^levels base products instead of 4^levels.  In a ragged
// batch every instance keeps its own sizes at every level (h follows its own
// n), so the work follows the instance, not the size class's largest.
//
// Memory, per top-level instance: level j (1 .. levels) holds 3^j operand
// slots of hmax_j words (the level size of the batch's largest instance) for
// a and for b (children 3 q, 3 q + 1, 3 q + 2 of parent q are x0, x1 and
// |x0 - x1|), their products (2 hmax_j words each) and one sign byte per
// parent and operand.  Both kernels keep their data in registers, one 4-word
// chunk per lane and row, and add with the workgroup ballot adder after a
// single barrier:
//   kara_split_kernel    one workgroup per (parent, operand): loads x0 and
//                        x1, stores them as the first two children, and
//                        forms x0 + ~x1 + 1 and x1 + ~x0 + 1 together; the
//                        carry out of the first (x0 >= x1) picks |x0 - x1|
//                        and gives the sign.
//   kara_combine_kernel  one workgroup per parent: the biased column sum
//                        V_k = (the five terms above at word k) + 2^63 -
//                        2^31 [k > 0] is unsigned, and the biases sum to
//                        2^31 2^(32 W), beyond the W result words; the low
//                        word of V_k and the high word of V_(k-1) are the
//                        two addends at word k.
#include <algorithm>
#include <atomic>

#include "bi_common.hpp"
#include "bi_internal.hpp"
#include "bi_wgadd.hpp"

namespace bi {

namespace {

__host__ __device__ inline uint32_t kara_half(uint32_t n) { return ((n + 1) / 2 + 3) & ~3u; }

// Instance count of a launch: a host value, or a device word times a factor
// (ragged lists, whose counts are known only on the device).
struct CountRef {
    const uint32_t *ptr;
    uint64_t mult, host;
    __device__ __forceinline__ uint64_t get() const { return ptr ? uint64_t(*ptr) * mult : host; }
};

// Operands of level j >= 1: instance q in slots of `stride` words at a and b
// (product at c, 2 stride words per slot).  Its size is `stride` (uniform
// batch), or for a ragged one the level-j size of its top-level instance
// q / 3^j, whose size top_n holds.
struct LevelInst {
    const uint32_t *a, *b;
    uint32_t *c;
    uint32_t stride, j;
    const uint32_t *top_n;
    uint64_t div;  // 3^j
    CountRef cnt;
    __device__ __forceinline__ uint64_t count() const { return cnt.get(); }
    __device__ __forceinline__ InstRef get(uint64_t q) const {
        uint32_t n = stride;
        if (top_n) {
            n = top_n[q / div];
            for (uint32_t i = 0; i < j; ++i) n = kara_half(n);
        }
        return InstRef{a + q * stride, b + q * stride, c + q * 2 * stride, n};
    }
};

// Instances [base, base + chunk) of a ragged size-class list.
struct ListChunk {
    ListInst src;
    uint64_t base, chunk;
    __device__ __forceinline__ uint64_t count() const {
        const uint64_t c = src.count();
        return c > base ? min(c - base, chunk) : 0;
    }
    __device__ __forceinline__ InstRef get(uint64_t q) const { return src.get(base + q); }
};

// Where the last level's split publishes its children for a base launch over
// a ragged list (descriptors, identity list, count); desc is null otherwise.
struct BaseList {
    bi_desc *desc;
    uint32_t *list;
    uint32_t *count;
};

__device__ __forceinline__ uint4 ld4(const uint32_t *p) { return *reinterpret_cast<const uint4 *>(p); }

// Words k .. k+3 of x (n words, zero beyond).
__device__ __forceinline__ void load_chunk(const uint32_t *x, uint32_t n, uint32_t k, bool vec, uint32_t (&v)[4]) {
    if (vec && k + 4 <= n) {
        const uint4 t = ld4(x + k);
        v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
    } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) v[t] = k + uint32_t(t) < n ? x[k + t] : 0u;
    }
}

__device__ __forceinline__ void store_chunk(uint32_t *p, const uint32_t (&v)[4]) {
    *reinterpret_cast<uint4 *>(p) = make_uint4(v[0], v[1], v[2], v[3]);
}

// Parent q of src (n words, split at h = kara_half(n)) into child slots of
// hs words at xa / xb + 3 q hs.  Wave w holds rows w R .. w R + R - 1 of the
// h-word halves (4 words per lane and row).
template <int NW, int R, class Src>
__global__ __launch_bounds__(NW * 64) void kara_split_kernel(Src src, uint32_t hs, uint32_t *__restrict__ xa,
                                                               uint32_t *__restrict__ xb, uint8_t *__restrict__ sg,
                                                               uint32_t *cnt_out, uint32_t *n_out, BaseList bl) {
    __shared__ uint32_t summary[NW];
    const uint64_t cnt = src.count();
    const uint64_t q = blockIdx.x;
    const uint32_t op = blockIdx.y;
    if (q == 0 && op == 0 && threadIdx.x == 0) {
        if (cnt_out) *cnt_out = uint32_t(cnt);
        if (bl.count) *bl.count = uint32_t(3 * cnt);
    }
    if (q >= cnt) return;  // uniform across the workgroup
    const InstRef in = src.get(q);
    const uint32_t n = in.n, h = kara_half(n), nchunks = h / 4;
    if (n_out && op == 0 && threadIdx.x == 0) n_out[q] = n;
    if (bl.desc && op == 0 && threadIdx.x < 3) {
        const uint64_t child = 3 * q + threadIdx.x;
        bi_desc d;
        d.a_off = child * hs;
        d.b_off = child * hs;
        d.out_off = child * 2 * hs;
        d.n_limbs = h;
        d.reserved = 0;
        bl.desc[child] = d;
        bl.list[child] = uint32_t(child);
    }
    const uint32_t *x = op ? in.b : in.a;
    uint32_t *dst = (op ? xb : xa) + 3 * q * hs;
    const uint32_t lane = lane_id(), w = wave_in_block();
    const bool vec = (reinterpret_cast<uintptr_t>(x) & 15) == 0;  // h is a multiple of 4
    uint32_t lo[R][4], hi[R][4];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const uint32_t k = 4 * (64 * (w * R + uint32_t(i)) + lane);
        if (k < h) {
            load_chunk(x, n, k, vec, lo[i]);
            load_chunk(x, n, h + k, vec, hi[i]);
        } else {
#pragma unroll
            for (int t = 0; t < 4; ++t) lo[i][t] = hi[i][t] = 0;
        }
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const uint32_t k = 4 * (64 * (w * R + uint32_t(i)) + lane);
        if (k < h) {
            store_chunk(dst + k, lo[i]);
            store_chunk(dst + hs + k, hi[i]);
        }
    }
    // d1 = x0 + ~x1 + 1 and d2 = x1 + ~x0 + 1 (mod 2^(32 h)), side by side
    uint32_t s1[R][4], s2[R][4], valid[R];
    uint64_t G1[R], P1[R], G2[R], P2[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const uint32_t r = w * R + uint32_t(i), c = 64 * r + lane;
        const bool in_range = c < nchunks;
        valid[i] = nchunks > 64 * r ? min(nchunks - 64 * r, 64u) : 0u;
        uint32_t nhi[4], nlo[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            nhi[t] = in_range ? ~hi[i][t] : 0u;
            nlo[t] = in_range ? ~lo[i][t] : 0u;
        }
        const uint32_t g1 = add_words<4>(lo[i], nhi, s1[i]);
        const uint32_t g2 = add_words<4>(hi[i], nlo, s2[i]);
        G1[i] = ballot(in_range && g1);
        P1[i] = ballot(in_range && all_ones<4>(s1[i]));
        G2[i] = ballot(in_range && g2);
        P2[i] = ballot(in_range && all_ones<4>(s2[i]));
    }
    uint32_t c1 = w == 0 ? 1u : 0u, c2 = c1, p1 = 1, p2 = 1;
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const uint32_t v = valid[i];
        const uint64_t vmask = v >= 64 ? ~0ull : ((1ull << v) - 1);
        const WaveCarry w1 = wave_carry(G1[i], P1[i], c1), w2 = wave_carry(G2[i], P2[i], c2);
        c1 = v >= 64 ? w1.out : uint32_t(w1.into >> v) & 1u;
        c2 = v >= 64 ? w2.out : uint32_t(w2.into >> v) & 1u;
        p1 &= P1[i] == vmask ? 1u : 0u;
        p2 &= P2[i] == vmask ? 1u : 0u;
    }
    if (lane == 0) summary[w] = c1 | (p1 << 1) | (c2 << 2) | (p2 << 3);
    __syncthreads();
    uint32_t in1 = 0, in2 = 0, t1 = 0;
    for (uint32_t v = 0; v < uint32_t(NW); ++v) {
        const uint32_t sv = summary[v];
        if (v < w) {
            in1 = (sv & 1u) | ((sv >> 1) & in1);
            in2 = ((sv >> 2) & 1u) | ((sv >> 3) & in2);
        }
        t1 = (sv & 1u) | ((sv >> 1) & t1);
    }
    if (w == 0) in1 = in2 = 1;
    const bool ge = t1 != 0;  // no borrow out of x0 - x1: x0 >= x1
    if (threadIdx.x == 0) sg[2 * q + op] = uint8_t(ge ? 0 : 1);
    uint32_t cin = ge ? in1 : in2;
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const uint32_t c = 64 * (w * R + uint32_t(i)) + lane;
        const WaveCarry wc = ge ? wave_carry(G1[i], P1[i], cin) : wave_carry(G2[i], P2[i], cin);
        uint32_t d[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) d[t] = ge ? s1[i][t] : s2[i][t];
        add_carry_words<4>(d, uint32_t(wc.into >> lane) & 1u);
        const uint32_t v = valid[i];
        cin = v >= 64 ? wc.out : uint32_t(wc.into >> v) & 1u;
        if (c < nchunks) store_chunk(dst + 2 * hs + 4 * c, d);
    }
}

// Parent q of Dst (n words; result 2 n words at c) from its children's
// products in slots of 2 hs words at z + 3 q (2 hs) (z0, z2, D in that order;
// the children have h = kara_half(n) words) and the sign bytes sg[2 q],
// sg[2 q + 1].  Wave w holds rows w R .. w R + R - 1 of the result.
template <int NW, int R, class Dst>
__global__ __launch_bounds__(NW * 64) void kara_combine_kernel(Dst dst, const uint32_t *__restrict__ z,
                                                                 const uint8_t *__restrict__ sg, uint32_t hs) {
    __shared__ uint32_t summary[NW];
    const uint64_t q = blockIdx.x;
    if (q >= dst.count()) return;
    const InstRef o = dst.get(q);
    const uint32_t W = 2 * o.n, h = kara_half(o.n);  // W <= 4 h
    const uint32_t *z0 = z + 3 * q * 2 * hs, *z2 = z0 + 2 * hs, *dv = z2 + 2 * hs;
    const uint32_t lane = lane_id(), w = wave_in_block();
    constexpr uint64_t kBias = uint64_t(1) << 63;
    // Every read first, so that they overlap: per row the chunk's z0 / z2
    // words and, inside the middle band [h, 3 h), z0, z2 and D at k0 - h
    // (addresses outside the chunk's regions are clamped into the slots and
    // their words unused); and for lane 0 of the wave's first row the terms
    // of the word below it, the wave below's last word.
    const uint8_t sgn0 = sg[2 * q], sgn1 = sg[2 * q + 1];
    uint4 A[R], Bm[R], Cm[R], Dm[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const uint32_t k0 = 4 * (64 * (w * R + uint32_t(i)) + lane);
        const uint32_t ka = k0 < W ? k0 : 0u;  // k0 + 3 < 4 h; h is a multiple of 4: one region per chunk
        const uint32_t m = k0 >= h && k0 < 3 * h && k0 < W ? k0 - h : 0u;
        A[i] = ka < 2 * h ? ld4(z0 + ka) : ld4(z2 + (ka - 2 * h));
        Bm[i] = ld4(z0 + m);
        Cm[i] = ld4(z2 + m);
        Dm[i] = ld4(dv + m);
    }
    const uint32_t kb = lane == 0 && w > 0 ? 256 * w * R - 1 : 0u;  // < W: the rows below hold words
    const bool bmid = kb >= h && kb < 3 * h;
    const uint32_t mb = bmid ? kb - h : 0u;
    const uint32_t eb0 = kb < 2 * h ? z0[kb] : z2[kb - 2 * h], eb1 = z0[mb], eb2 = z2[mb], eb3 = dv[mb];
    const bool sub = sgn0 == sgn1;
    uint32_t xs[R][4], ys[R][4];
    uint32_t top_prev = 0;  // high word of the previous row's last V (lane 63)
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const uint32_t k0 = 4 * (64 * (w * R + uint32_t(i)) + lane);
        uint64_t V[4] = {kBias + A[i].x, kBias + A[i].y, kBias + A[i].z, kBias + A[i].w};
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if (k0 + t > 0) V[t] -= uint64_t(1) << 31;
        if (k0 >= h && k0 < 3 * h) {
            V[0] += uint64_t(Bm[i].x) + Cm[i].x;
            V[1] += uint64_t(Bm[i].y) + Cm[i].y;
            V[2] += uint64_t(Bm[i].z) + Cm[i].z;
            V[3] += uint64_t(Bm[i].w) + Cm[i].w;
            if (sub) {
                V[0] -= Dm[i].x; V[1] -= Dm[i].y; V[2] -= Dm[i].z; V[3] -= Dm[i].w;
            } else {
                V[0] += Dm[i].x; V[1] += Dm[i].y; V[2] += Dm[i].z; V[3] += Dm[i].w;
            }
        }
        // high word of V_(k0 - 1): the lane below; at lane 0 the previous
        // row's lane 63, or for the wave's first row the word recomputed
        uint32_t below = __shfl_up(uint32_t(V[3] >> 32), 1);
        if (lane == 0) {
            if (i > 0) {
                below = top_prev;
            } else if (kb > 0) {
                uint64_t v = kBias - (uint64_t(1) << 31) + eb0;
                if (bmid) {
                    v += uint64_t(eb1) + eb2;
                    v = sub ? v - eb3 : v + eb3;
                }
                below = uint32_t(v >> 32);
            } else {
                below = 0u;
            }
        }
        top_prev = __builtin_amdgcn_readlane(uint32_t(V[3] >> 32), 63);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const bool in = k0 + uint32_t(t) < W;
            xs[i][t] = in ? uint32_t(V[t]) : 0u;
            const uint32_t prev = t == 0 ? below : uint32_t(V[t - 1] >> 32);
            ys[i][t] = in && k0 + uint32_t(t) > 0 ? prev : 0u;
        }
    }
    const GlobalSink sink{o.c, W, (reinterpret_cast<uintptr_t>(o.c) & 15) == 0};
    (void)wg_add_regs<NW, R>(xs, ys, W, sink, summary);
}

// (waves, rows per wave) for an addition over `words` words: rows of 256
// words, one per wave up to 8 waves, then 2 per wave on 8 or 16 waves, then
// 4 (512-thread workgroups up to 16 rows keep four workgroups per CU).
struct Shape {
    int nw, r;
};
Shape kara_shape(uint32_t words) {
    const uint32_t rows = (words + 255) / 256;
    if (rows > 32) return {16, 4};
    if (rows > 16) return {16, 2};
    if (rows > 8) return {8, 2};
    return {rows > 4 ? 8 : rows > 2 ? 4 : rows > 1 ? 2 : 1, 1};
}

template <int NW, int R, class Src>
hipError_t launch_split_shape(const Src &src, uint64_t grid, uint32_t hs, uint32_t *xa, uint32_t *xb, uint8_t *sg,
                              uint32_t *cnt_out, uint32_t *n_out, const BaseList &bl, hipStream_t st) {
    hipLaunchKernelGGL((kara_split_kernel<NW, R, Src>), dim3(uint32_t(grid), 2), dim3(NW * 64), 0, st, src, hs, xa, xb,
                       sg, cnt_out, n_out, bl);
    return hipGetLastError();
}

// Split of `grid` parents into child slots of hs words (the largest child).
template <class Src>
hipError_t launch_split(const Src &src, uint64_t grid, uint32_t hs, uint32_t *xa, uint32_t *xb, uint8_t *sg,
                        uint32_t *cnt_out, uint32_t *n_out, const BaseList &bl, hipStream_t st) {
    if (grid == 0) return hipSuccess;
    const Shape sh = kara_shape(hs);
#define BI_KARA_SPLIT(NW_, R_) \
    if (sh.nw == NW_ && sh.r == R_) return launch_split_shape<NW_, R_>(src, grid, hs, xa, xb, sg, cnt_out, n_out, bl, st);
    BI_KARA_SPLIT(1, 1) BI_KARA_SPLIT(2, 1) BI_KARA_SPLIT(4, 1) BI_KARA_SPLIT(8, 1) BI_KARA_SPLIT(8, 2)
    BI_KARA_SPLIT(16, 2) BI_KARA_SPLIT(16, 4)
#undef BI_KARA_SPLIT
    return hipErrorInvalidValue;
}

template <int NW, int R, class Dst>
hipError_t launch_combine_shape(const Dst &dst, uint64_t grid, const uint32_t *z, const uint8_t *sg, uint32_t hs,
                                hipStream_t st) {
    hipLaunchKernelGGL((kara_combine_kernel<NW, R, Dst>), dim3(uint32_t(grid)), dim3(NW * 64), 0, st, dst, z, sg, hs);
    return hipGetLastError();
}

// Combine of `grid` parents of at most nparent words from child slots of hs words.
template <class Dst>
hipError_t launch_combine(const Dst &dst, uint32_t nparent, uint64_t grid, const uint32_t *z, const uint8_t *sg,
                          uint32_t hs, hipStream_t st) {
    if (grid == 0) return hipSuccess;
    const Shape sh = kara_shape(2 * nparent);
#define BI_KARA_COMBINE(NW_, R_) \
    if (sh.nw == NW_ && sh.r == R_) return launch_combine_shape<NW_, R_>(dst, grid, z, sg, hs, st);
    BI_KARA_COMBINE(1, 1) BI_KARA_COMBINE(2, 1) BI_KARA_COMBINE(4, 1) BI_KARA_COMBINE(8, 1) BI_KARA_COMBINE(8, 2)
    BI_KARA_COMBINE(16, 2) BI_KARA_COMBINE(16, 4)
#undef BI_KARA_COMBINE
    return hipErrorInvalidValue;
}

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

uint64_t pow3(int j) {
    uint64_t r = 1;
    for (int i = 0; i < j; ++i) r *= 3;
    return r;
}

// Scratch of a round of R top-level instances: per level the operands, the
// products and the sign bytes; for ragged rounds the top-level sizes, the
// base list and the counts; then the base algorithm's own scratch.
struct KaraLayout {
    size_t xa[kKaraMaxLevels + 1], xb[kKaraMaxLevels + 1], z[kKaraMaxLevels + 1], sg[kKaraMaxLevels + 1];
    size_t topn, desc, list, counts, base, total;
};

KaraLayout kara_layout(const KaraPlan &p, uint64_t R, bool list, size_t base_bytes) {
    KaraLayout l{};
    size_t off = 0;
    for (int j = 1; j <= p.levels; ++j) {
        const uint64_t cj = R * pow3(j);
        l.xa[j] = off;
        off = al256(off + 4 * cj * p.h[j]);
        l.xb[j] = off;
        off = al256(off + 4 * cj * p.h[j]);
        l.z[j] = off;
        off = al256(off + 8 * cj * p.h[j]);
        l.sg[j] = off;
        off = al256(off + 2 * (cj / 3));
    }
    const uint64_t cl = R * pow3(p.levels);
    l.topn = off;
    if (list) off = al256(off + 4 * R);
    l.desc = off;
    if (list) off = al256(off + sizeof(bi_desc) * cl);
    l.list = off;
    if (list) off = al256(off + 4 * cl);
    l.counts = off;
    off = al256(off + 4 * (kKaraMaxLevels + 2));
    l.base = off;
    l.total = off + base_bytes;
    return l;
}

}  // namespace

KaraPlan kara_plan(uint32_t n32, uint32_t base) {
    KaraPlan p;
    p.h[0] = n32;
    uint32_t h = n32;
    do {
        h = kara_half(h);
        p.h[++p.levels] = h;
    } while (h > base && p.levels < kKaraMaxLevels);
    return p;
}

size_t kara_round_bytes(const KaraPlan &p, uint64_t R, bool list, size_t base_bytes) {
    return kara_layout(p, R, list, base_bytes).total;
}

// Levels 0 .. levels-1 split, the base products, then the combines back up.
// The top level's instances come from `top` (UniformInst or ListChunk) and its
// results go to top.get(q).c; lower levels live in the scratch.
template <class Top, class Base>
static bi_status kara_run(const Top &top, uint64_t grid0, const KaraPlan &p, uint8_t *scr, const KaraLayout &l,
                          bool list, Base &&base, hipStream_t st) {
    auto *counts = reinterpret_cast<uint32_t *>(scr + l.counts);
    auto P = [&](size_t off) { return reinterpret_cast<uint32_t *>(scr + off); };
    const BaseList none{nullptr, nullptr, nullptr};
    const BaseList bl{reinterpret_cast<bi_desc *>(scr + l.desc), P(l.list), counts + 1};
    // a device count (ragged rounds) or the host's
    auto cref = [&](int j) {
        return list ? CountRef{counts, pow3(j), 0} : CountRef{nullptr, 1, grid0 * pow3(j)};
    };
    // ragged rounds: every instance's own sizes, from its top-level size
    uint32_t *top_n = list ? P(l.topn) : nullptr;
    auto level = [&](uint32_t *a, uint32_t *b, uint32_t *c, int j) {
        return LevelInst{a, b, c, p.h[j], uint32_t(j), top_n, pow3(j), cref(j)};
    };
    hipError_t e = hipSuccess;
    for (int j = 0; j < p.levels && e == hipSuccess; ++j) {
        const BaseList &b = (list && j + 1 == p.levels) ? bl : none;
        uint8_t *sg = scr + l.sg[j + 1];
        if (j == 0)
            e = launch_split(top, grid0, p.h[1], P(l.xa[1]), P(l.xb[1]), sg, list ? counts : nullptr, top_n, b, st);
        else
            e = launch_split(level(P(l.xa[j]), P(l.xb[j]), nullptr, j), grid0 * pow3(j), p.h[j + 1], P(l.xa[j + 1]),
                             P(l.xb[j + 1]), sg, nullptr, nullptr, b, st);
    }
    if (e != hipSuccess) return set_error(BI_EHIP, "Karatsuba split launch: %s", hipGetErrorString(e));
    const int L = p.levels;
    const bi_status s = base(P(l.xa[L]), P(l.xb[L]), P(l.z[L]), p.h[L], grid0 * pow3(L), bl);
    if (s != BI_OK) return s;
    for (int j = L - 1; j >= 0 && e == hipSuccess; --j) {
        const uint8_t *sg = scr + l.sg[j + 1];
        if (j == 0)
            e = launch_combine(top, p.h[0], grid0, P(l.z[1]), sg, p.h[1], st);
        else
            e = launch_combine(level(nullptr, nullptr, P(l.z[j]), j), p.h[j], grid0 * pow3(j), P(l.z[j + 1]), sg,
                               p.h[j + 1], st);
    }
    if (e != hipSuccess) return set_error(BI_EHIP, "Karatsuba combine launch: %s", hipGetErrorString(e));
    return BI_OK;
}

bi_status launch_bigmul_kara(Ctx &c, const uint32_t *a, const uint32_t *b, uint32_t *out, uint32_t n32,
                             uint64_t batch, const KaraPlan &p, int base_algo, size_t base_bytes, uint8_t *scr,
                             uint64_t round, hipStream_t st) {
    if (batch == 0) return BI_OK;
    if (round == 0) return set_error(BI_ESIZE, "Karatsuba scratch holds no instance");
    for (uint64_t b0 = 0; b0 < batch; b0 += round) {
        const uint64_t R = std::min(round, batch - b0);
        const KaraLayout l = kara_layout(p, R, false, base_bytes);
        const UniformInst top{a + b0 * n32, b + b0 * n32, out + b0 * 2 * n32, n32, R};
        auto base = [&](const uint32_t *A, const uint32_t *B, uint32_t *C, uint32_t h, uint64_t cnt,
                        const BaseList &) {
            return dispatch_bigmul(c, A, B, C, h, cnt, base_algo, st, base_bytes ? scr + l.base : nullptr,
                                   base_bytes);
        };
        const bi_status s = kara_run(top, R, p, scr, l, false, base, st);
        if (s != BI_OK) return s;
    }
    return BI_OK;
}

hipError_t launch_bigmul_kara_list(const Ctx &c, const Tune &tune, const ListInst &src, uint32_t nmax,
                                   uint64_t count_max, uint8_t *scr, size_t scr_bytes, hipStream_t st) {
    const KaraPlan p = kara_plan_tuned(tune, nmax);
    const int L = p.levels;
    const int alg = kara_base_algo(tune, p.h[L], true);
    // rounds of as many instances as the scratch holds with the base's list scratch
    uint64_t R = std::max<uint64_t>(1, std::min<uint64_t>(count_max, kKaraListRound));
    while (R > 1 && kara_round_bytes(p, R, true, list_algo_scratch_bytes(alg, p.h[L], R * pow3(L))) > scr_bytes)
        R /= 2;
    const size_t base_bytes = list_algo_scratch_bytes(alg, p.h[L], R * pow3(L));
    const KaraLayout l = kara_layout(p, R, true, base_bytes);
    if (l.total > scr_bytes) return hipErrorInvalidValue;
    for (uint64_t b0 = 0; b0 < count_max; b0 += R) {
        const ListChunk top{src, b0, R};
        hipError_t he = hipSuccess;
        auto base = [&](const uint32_t *A, const uint32_t *B, uint32_t *C, uint32_t h, uint64_t cnt,
                        const BaseList &bl) {
            const ListInst in{A, B, C, bl.desc, bl.list, bl.count, 1};
            he = launch_bigmul_list_algo(c, tune, in, h, cnt, alg, base_bytes ? scr + l.base : nullptr, base_bytes, st);
            return he == hipSuccess ? BI_OK : BI_EHIP;
        };
        const bi_status s = kara_run(top, R, p, scr, l, true, base, st);
        if (s != BI_OK) return he != hipSuccess ? he : hipErrorLaunchFailure;
    }
    return hipSuccess;
}

size_t kara_list_scratch_bound(uint64_t count) {
    // the largest class, for each base size the tuning may choose: full
    // rounds with a base that needs no scratch (the schoolbook kernels), or
    // rounds of one instance with the largest base scratch any algorithm
    // takes (launch_bigmul_kara_list shrinks its rounds to fit)
    size_t bound = 0;
    for (uint32_t b : kKaraBases) {
        const KaraPlan p = kara_plan(kMaxLimbs32, b);
        const uint64_t R = std::max<uint64_t>(1, std::min<uint64_t>(count, kKaraListRound));
        size_t base = 0;
        for (int alg : {BI_MUL_SCHOOL_VALU, BI_MUL_SCHOOL_MFMA, BI_MUL_NTT, BI_MUL_NTT_PF64})
            base = std::max(base, list_algo_scratch_bytes(alg, p.h[p.levels], pow3(p.levels)));
        bound = std::max({bound, kara_round_bytes(p, R, true, 0), kara_round_bytes(p, 1, true, base)});
    }
    return bound;
}

}  // namespace bi
