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
// so a pair costs 3^levels base products instead of 4^levels.
//
// Memory, per top-level instance: level j (1 .. levels) holds 3^j operands of
// h_j words for a and for b (children 3 q, 3 q + 1, 3 q + 2 of parent q are
// x0, x1 and |x0 - x1|), their products (2 h_j words each) and one sign byte
// per parent and operand.
//   kara_split_kernel    one workgroup per (parent, operand): stages the
//                        parent's words [0, 2 h) (zero beyond its length) in
//                        LDS and writes them out as x0 | x1, finds the highest
//                        word where x0 and x1 differ (the sign), and writes
//                        |x0 - x1| = big + ~small + 1 with the workgroup
//                        ballot adder.
//   kara_combine_kernel  one workgroup per parent: the biased column sum
//                        V_k = (the five terms above at word k) + 2^63 -
//                        2^31 [k > 0] is unsigned, and the biases sum to
//                        2^31 2^(32 W), beyond the W result words; the low
//                        words of all V_k and their high words are staged
//                        in LDS, and the ballot adder writes
//                        sum_k lo(V_k) 2^(32 k) + hi(V_k) 2^(32 (k+1)).
#include <algorithm>
#include <atomic>

#include "bi_common.hpp"
#include "bi_internal.hpp"
#include "bi_wgadd.hpp"

namespace bi {

namespace {

// Instance count of a launch: a host value, or a device word times a factor
// (ragged lists, whose counts are known only on the device).
struct CountRef {
    const uint32_t *ptr;
    uint64_t mult, host;
    __device__ __forceinline__ uint64_t get() const { return ptr ? uint64_t(*ptr) * mult : host; }
};

// Operands of a level below the top: instance q at a + q n and b + q n; its
// product at c + 2 q n.
struct LevelInst {
    const uint32_t *a, *b;
    uint32_t *c;
    uint32_t n;
    CountRef cnt;
    __device__ __forceinline__ uint64_t count() const { return cnt.get(); }
    __device__ __forceinline__ InstRef get(uint64_t q) const {
        return InstRef{a + q * n, b + q * n, c + q * 2 * n, n};
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

template <int NW, class Src>
__global__ __launch_bounds__(NW * 64) void kara_split_kernel(Src src, uint32_t h, uint32_t *__restrict__ xa,
                                                               uint32_t *__restrict__ xb, uint8_t *__restrict__ sg,
                                                               uint32_t *cnt_out, BaseList bl) {
    extern __shared__ __align__(16) uint32_t sh[];  // 2 h staged words, then NW summary words
    __shared__ uint32_t top;
    constexpr uint32_t T = NW * 64;
    const uint64_t cnt = src.count();
    const uint64_t q = blockIdx.x;
    const uint32_t op = blockIdx.y;
    if (q == 0 && op == 0 && threadIdx.x == 0) {
        if (cnt_out) *cnt_out = uint32_t(cnt);
        if (bl.count) *bl.count = uint32_t(3 * cnt);
    }
    if (q >= cnt) return;  // uniform across the workgroup
    const InstRef in = src.get(q);
    const uint32_t *x = op ? in.b : in.a;
    const uint32_t n = in.n;
    uint32_t *dst = (op ? xb : xa) + 3 * q * h;
    // x0 | x1 = the parent's words [0, 2 h), zero beyond its length: U
    // 16-byte groups per thread loaded before any is stored, so several
    // loads are in flight
    const bool vec = (reinterpret_cast<uintptr_t>(x) & 15) == 0;
    const uint32_t ng = h / 2;  // 16-byte groups in 2 h words
    constexpr int U = 4;
    for (uint32_t g0 = threadIdx.x; g0 < ng; g0 += U * T) {
        uint4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t w = 4 * (g0 + u * T);
            if (vec && w + 4 <= n) {
                v[u] = ld4(x + w);
            } else {
                v[u].x = w < n ? x[w] : 0u;
                v[u].y = w + 1 < n ? x[w + 1] : 0u;
                v[u].z = w + 2 < n ? x[w + 2] : 0u;
                v[u].w = w + 3 < n ? x[w + 3] : 0u;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t g = g0 + u * T;
            if (g < ng) {
                *reinterpret_cast<uint4 *>(sh + 4 * g) = v[u];
                *reinterpret_cast<uint4 *>(dst + 4 * g) = v[u];
            }
        }
    }
    if (threadIdx.x == 0) top = 0;
    __syncthreads();
    uint32_t hi = 0;  // 1 + the highest word index where x0 and x1 differ (0: none)
    for (uint32_t w = threadIdx.x; w < h; w += T)
        if (sh[w] != sh[h + w]) hi = w + 1;
    if (hi) atomicMax(&top, hi);
    __syncthreads();
    const uint32_t t = top;
    const uint32_t less = t && sh[t - 1] < sh[h + t - 1] ? 1u : 0u;  // x0 < x1
    if (threadIdx.x == 0) sg[2 * q + op] = uint8_t(less);
    if (bl.desc && op == 0 && threadIdx.x < 3) {
        const uint64_t child = 3 * q + threadIdx.x;
        bi_desc d;
        d.a_off = child * h;
        d.b_off = child * h;
        d.out_off = child * 2 * h;
        d.n_limbs = h;
        d.reserved = 0;
        bl.desc[child] = d;
        bl.list[child] = uint32_t(child);
    }
    // |x0 - x1| = big + ~small + 1 mod 2^(32 h); h is a multiple of 4
    const uint32_t *big = sh + (less ? h : 0), *small = sh + (less ? 0 : h);
    auto terms = [&](uint32_t c, uint32_t (&u)[4], uint32_t (&v)[4]) {
        const uint4 bb = ld4(big + 4 * c), ss = ld4(small + 4 * c);
        u[0] = bb.x; u[1] = bb.y; u[2] = bb.z; u[3] = bb.w;
        v[0] = ~ss.x; v[1] = ~ss.y; v[2] = ~ss.z; v[3] = ~ss.w;
    };
    uint32_t *dd = dst + 2 * h;
    const GlobalSink sink{dd, h, (reinterpret_cast<uintptr_t>(dd) & 15) == 0};
    (void)wg_add_rows_sink<NW>(terms, sink, h, sh + 2 * h, 1u);
}

// Parent q of Dst (result words 2 n at c) from its children's products at
// z + 3 q (2 h) (z0, z2, D in that order) and the sign bytes sg[2 q], sg[2 q + 1].
// The column sums of every word go to LDS first (low words at Ls[k], high
// words at Hs[k]; 4 h words each), then the ballot adder adds Ls + Hs
// shifted by one word.
template <int NW, class Dst>
__global__ __launch_bounds__(NW * 64) void kara_combine_kernel(Dst dst, const uint32_t *__restrict__ z,
                                                                 const uint8_t *__restrict__ sg, uint32_t h) {
    extern __shared__ __align__(16) uint32_t sh[];  // Ls (4 h), Hs (4 h), NW summary words
    constexpr uint32_t T = NW * 64;
    const uint64_t q = blockIdx.x;
    if (q >= dst.count()) return;
    const InstRef o = dst.get(q);
    const uint32_t W = 2 * o.n;  // result words, at most 4 h
    const uint32_t *z0 = z + 3 * q * 2 * h, *z2 = z0 + 2 * h, *dv = z2 + 2 * h;
    const bool sub = sg[2 * q] == sg[2 * q + 1];
    uint32_t *Ls = sh, *Hs = sh + 4 * h, *summary = sh + 8 * h;
    constexpr uint64_t kBias = uint64_t(1) << 63;
    const uint32_t nchunks = (W + 3) / 4;
    constexpr int U = 2;
    for (uint32_t c0 = threadIdx.x; c0 < nchunks; c0 += U * T) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t c = c0 + u * T;
            if (c >= nchunks) break;
            const uint32_t k0 = 4 * c;  // < 4 h; h is a multiple of 4, so the chunk lies in one region
            const uint4 A = k0 < 2 * h ? ld4(z0 + k0) : ld4(z2 + (k0 - 2 * h));
            uint64_t V[4] = {kBias + A.x, kBias + A.y, kBias + A.z, kBias + A.w};
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (k0 + t > 0) V[t] -= uint64_t(1) << 31;
            if (k0 >= h && k0 < 3 * h) {
                const uint32_t m = k0 - h;
                const uint4 B = ld4(z0 + m), C = ld4(z2 + m), Dd = ld4(dv + m);
                V[0] += uint64_t(B.x) + C.x;
                V[1] += uint64_t(B.y) + C.y;
                V[2] += uint64_t(B.z) + C.z;
                V[3] += uint64_t(B.w) + C.w;
                if (sub) {
                    V[0] -= Dd.x; V[1] -= Dd.y; V[2] -= Dd.z; V[3] -= Dd.w;
                } else {
                    V[0] += Dd.x; V[1] += Dd.y; V[2] += Dd.z; V[3] += Dd.w;
                }
            }
            *reinterpret_cast<uint4 *>(Ls + k0) =
                make_uint4(uint32_t(V[0]), uint32_t(V[1]), uint32_t(V[2]), uint32_t(V[3]));
            *reinterpret_cast<uint4 *>(Hs + k0) = make_uint4(uint32_t(V[0] >> 32), uint32_t(V[1] >> 32),
                                                             uint32_t(V[2] >> 32), uint32_t(V[3] >> 32));
        }
    }
    __syncthreads();
    auto terms = [&](uint32_t c, uint32_t (&x)[4], uint32_t (&y)[4]) {
        const uint32_t k0 = 4 * c;
        const uint4 l = ld4(Ls + k0);
        x[0] = l.x; x[1] = l.y; x[2] = l.z; x[3] = l.w;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const uint32_t k = k0 + t;
            if (k >= W) x[t] = 0;
            y[t] = k > 0 && k < W ? Hs[k - 1] : 0u;
        }
    };
    const GlobalSink sink{o.c, W, (reinterpret_cast<uintptr_t>(o.c) & 15) == 0};
    (void)wg_add_rows_sink<NW>(terms, sink, W, summary);
}

// Waves per workgroup for an addition of `words` words: one row of 256 words
// per wave, 1 to 16 waves.
int kara_waves(uint32_t words) {
    const uint32_t rows = (words + 255) / 256;
    return rows >= 16 ? 16 : rows >= 8 ? 8 : rows >= 4 ? 4 : rows >= 2 ? 2 : 1;
}

template <int NW, class Src>
hipError_t launch_split_nw(const Src &src, uint64_t grid, uint32_t h, uint32_t *xa, uint32_t *xb, uint8_t *sg,
                           uint32_t *cnt_out, const BaseList &bl, hipStream_t st) {
    const size_t lds = sizeof(uint32_t) * (2 * size_t(h) + NW);
    hipLaunchKernelGGL((kara_split_kernel<NW, Src>), dim3(uint32_t(grid), 2), dim3(NW * 64), lds, st, src, h, xa, xb,
                       sg, cnt_out, bl);
    return hipGetLastError();
}

// Split of `grid` parents into children of h words (the subtraction adds h words).
template <class Src>
hipError_t launch_split(const Src &src, uint64_t grid, uint32_t h, uint32_t *xa, uint32_t *xb, uint8_t *sg,
                        uint32_t *cnt_out, const BaseList &bl, hipStream_t st) {
    if (grid == 0) return hipSuccess;
    switch (kara_waves(h)) {
        case 16: return launch_split_nw<16>(src, grid, h, xa, xb, sg, cnt_out, bl, st);
        case 8: return launch_split_nw<8>(src, grid, h, xa, xb, sg, cnt_out, bl, st);
        case 4: return launch_split_nw<4>(src, grid, h, xa, xb, sg, cnt_out, bl, st);
        case 2: return launch_split_nw<2>(src, grid, h, xa, xb, sg, cnt_out, bl, st);
        default: return launch_split_nw<1>(src, grid, h, xa, xb, sg, cnt_out, bl, st);
    }
}

template <int NW, class Dst>
hipError_t launch_combine_nw(const Dst &dst, uint64_t grid, const uint32_t *z, const uint8_t *sg, uint32_t h,
                             hipStream_t st) {
    const size_t lds = sizeof(uint32_t) * (8 * size_t(h) + NW);
    static std::atomic<uint64_t> lds_set{0};  // up to 128 KiB at 4096-word children
    const hipError_t e = lds_limit_once(reinterpret_cast<const void *>(&kara_combine_kernel<NW, Dst>), lds_set);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((kara_combine_kernel<NW, Dst>), dim3(uint32_t(grid)), dim3(NW * 64), lds, st, dst, z, sg, h);
    return hipGetLastError();
}

// Combine of `grid` parents of nparent words from children of h words.
template <class Dst>
hipError_t launch_combine(const Dst &dst, uint32_t nparent, uint64_t grid, const uint32_t *z, const uint8_t *sg,
                          uint32_t h, hipStream_t st) {
    if (grid == 0) return hipSuccess;
    switch (kara_waves(2 * nparent)) {
        case 16: return launch_combine_nw<16>(dst, grid, z, sg, h, st);
        case 8: return launch_combine_nw<8>(dst, grid, z, sg, h, st);
        case 4: return launch_combine_nw<4>(dst, grid, z, sg, h, st);
        case 2: return launch_combine_nw<2>(dst, grid, z, sg, h, st);
        default: return launch_combine_nw<1>(dst, grid, z, sg, h, st);
    }
}

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

uint64_t pow3(int j) {
    uint64_t r = 1;
    for (int i = 0; i < j; ++i) r *= 3;
    return r;
}

// Scratch of a round of R top-level instances: per level the operands, the
// products and the sign bytes; for ragged rounds the base list and the
// counts; then the base algorithm's own scratch.
struct KaraLayout {
    size_t xa[kKaraMaxLevels + 1], xb[kKaraMaxLevels + 1], z[kKaraMaxLevels + 1], sg[kKaraMaxLevels + 1];
    size_t desc, list, counts, base, total;
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
        h = ((h + 1) / 2 + 3) & ~3u;
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
    hipError_t e = hipSuccess;
    for (int j = 0; j < p.levels && e == hipSuccess; ++j) {
        const BaseList &b = (list && j + 1 == p.levels) ? bl : none;
        uint8_t *sg = scr + l.sg[j + 1];
        if (j == 0)
            e = launch_split(top, grid0, p.h[1], P(l.xa[1]), P(l.xb[1]), sg, list ? counts : nullptr, b, st);
        else
            e = launch_split(LevelInst{P(l.xa[j]), P(l.xb[j]), nullptr, p.h[j], cref(j)}, grid0 * pow3(j), p.h[j + 1],
                             P(l.xa[j + 1]), P(l.xb[j + 1]), sg, nullptr, b, st);
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
            e = launch_combine(LevelInst{nullptr, nullptr, P(l.z[j]), p.h[j], cref(j)}, p.h[j], grid0 * pow3(j),
                               P(l.z[j + 1]), sg, p.h[j + 1], st);
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
    const KaraPlan p = kara_plan(nmax, kKaraBase);
    const int L = p.levels;
    const int alg = kara_base_algo(tune, p.h[L]);
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
    // the largest class in full rounds with a base that needs no scratch (the
    // schoolbook kernels), or in rounds of one instance with the largest base
    // scratch any algorithm takes (launch_bigmul_kara_list shrinks its rounds
    // to fit)
    const KaraPlan p = kara_plan(kMaxLimbs32, kKaraBase);
    const uint64_t R = std::max<uint64_t>(1, std::min<uint64_t>(count, kKaraListRound));
    size_t base = 0;
    for (int alg : {BI_MUL_SCHOOL_VALU, BI_MUL_SCHOOL_MFMA, BI_MUL_NTT, BI_MUL_NTT_PF64})
        base = std::max(base, list_algo_scratch_bytes(alg, p.h[p.levels], pow3(p.levels)));
    return std::max(kara_round_bytes(p, R, true, 0), kara_round_bytes(p, 1, true, base));
}

}  // namespace bi
