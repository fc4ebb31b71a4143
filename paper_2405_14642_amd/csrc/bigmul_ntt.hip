// NTT multiplication (Section 4): number-theoretic transforms over two primes
// p < 2^31 with Chinese-remainder recombination, then carry normalisation.
//
// Operands are split into 16-bit coefficients (the 16-bit digits of the
// limbs), zero-padded to L = 2^M >= 2 * (number of coefficients) so the cyclic
// convolution does not wrap.  Per (pair, prime) one workgroup of L/32 threads:
//
//   forward DIF transform of a, forward DIF transform of b (natural order in,
//   bit-reversed order out, so no permutation step is needed), pointwise
//   Montgomery product, inverse DIT transform (bit-reversed in, natural out),
//   scaling by L^-1 (times 2^32 to undo the Montgomery factor).
//
// Each transform runs as three passes over the LDS-resident vector.  A pass
// covers R radix-2 stages at once: every thread loads 32 elements forming
// groups of 2^R, runs the 2^R-point DIF network in registers (twiddles are
// powers of the 2^R-th root, identical for all lanes, so they come through
// scalar loads), and multiplies output position k of a group by
// w^(2^s * lo * bitrev_R(k)) where lo is the group's offset (the four-step
// factorisation of the radix-2 stages of Fig. 8).  The inverse applies the
// inverse of each pass in reverse order.  LDS words are padded (one per 32)
// so that the strided element sets of all passes are bank-conflict free.
//
// A second kernel per pair recombines the two residues of every coefficient
// (Garner), folds each thread's 8 coefficients (16-bit positions) into 4 low
// words plus 2 high words, and adds the low and high arrays with the
// workgroup ballot-adder, as for the schoolbook product.
//
// The same transform code, templated over the field, runs the single-prime
// PrimeField64 variant of Section 4.1 (p = 29 2^57 + 1, 64-bit Montgomery
// multiplies).  One prime suffices for exactness, and instead of one transform
// of the zero-padded length L it runs two of length H = L/2: the cyclic
// convolution (c_lo + c_hi) and, on inputs twisted by powers of psi (psi^H =
// -1), the negacyclic one (c_lo - c_hi), where c = c_lo + x^H c_hi.  Every
// coefficient is below 2^46 < p, so (cyc + neg)/2 and (cyc - neg)/2 mod p are
// the coefficients themselves.
#include <algorithm>
#include <utility>

#include "bi_common.hpp"
#include "bi_internal.hpp"
#include "bi_wgadd.hpp"

namespace bi {

namespace {

constexpr int E = 32;  // elements per thread

__device__ __forceinline__ uint32_t add_mod(uint32_t a, uint32_t b, uint32_t p) {
    const uint32_t s = a + b;  // < 2p < 2^32
    return min(s, s - p);
}
__device__ __forceinline__ uint32_t sub_mod(uint32_t a, uint32_t b, uint32_t p) {
    const uint32_t d = a - b;
    return min(d, d + p);
}
// a * w mod p with the precomputed w' = floor(w 2^32 / p) (Shoup).
__device__ __forceinline__ uint32_t mul_shoup(uint32_t a, uint32_t w, uint32_t wsh, uint32_t p) {
    const uint32_t q = __umulhi(a, wsh);
    const uint32_t r = a * w - q * p;  // in [0, 2p)
    return min(r, r - p);
}
// a * b * 2^-32 mod p (Montgomery, pneg = -p^-1 mod 2^32).
__device__ __forceinline__ uint32_t mul_mont(uint32_t a, uint32_t b, uint32_t p, uint32_t pneg) {
    const uint64_t t = uint64_t(a) * b;
    const uint32_t tl = uint32_t(t), th = uint32_t(t >> 32);
    const uint32_t m = tl * pneg;
    const uint32_t u = th + __umulhi(m, p) + (tl != 0u ? 1u : 0u);  // < 2p
    return min(u, u - p);
}

// a * b * 2^-64 mod p for p = 29 2^57 + 1 (a, b < p).  -p^-1 mod 2^64 is
// 29 2^57 - 1 because p = 1 mod 2^57, so both the Montgomery factor m and the
// product m p reduce to shifts and a multiply by 29.
__device__ __forceinline__ uint64_t mul_mont64(uint64_t a, uint64_t b) {
    const uint64_t tl = a * b, th = __umul64hi(a, b);
    const uint64_t m = ((tl * 29u) << 57) - tl;            // tl (-p^-1) mod 2^64
    const uint64_t m29l = m * 29u, m29h = __umul64hi(m, 29u);
    const uint64_t mpl = m + (m29l << 57);                  // low word of m p = m + 29 m 2^57
    const uint64_t mph = ((m29h << 57) | (m29l >> 7)) + (mpl < m ? 1u : 0u);
    const uint64_t u = th + mph + (tl != 0 ? 1u : 0u);      // (a b + m p) / 2^64 < 2p
    return u >= kP64 ? u - kP64 : u;
}

// Field policies of the transform code: element type T, twiddle entry W, the
// tables' root order 2^kLogTab with their pass-table offsets, and how many
// butterflies (kBfly, 0 = a whole stage) and twiddle products (kTw, 0 = the
// default) the scheduler may interleave, which bounds live registers.
struct Fp32 {  // one prime below 2^31; twiddles (w, Shoup companion)
    using T = uint32_t;
    using W = uint2;
    static constexpr int kBfly = 0, kTw = 0;
    static constexpr int kLogTab = kNttLogLmax;
    static constexpr uint32_t kT1 = kNttT1;
    __device__ static constexpr uint32_t t0(uint32_t m) { return ntt_t0_offset(m); }
    uint32_t p;
    __device__ __forceinline__ T add(T a, T b) const { return add_mod(a, b, p); }
    __device__ __forceinline__ T sub(T a, T b) const { return sub_mod(a, b, p); }
    __device__ __forceinline__ T mulw(T a, W w) const { return mul_shoup(a, w.x, w.y, p); }
};
struct Fp64 {  // PrimeField64; twiddles in Montgomery form
    using T = uint64_t;
    using W = uint64_t;
    static constexpr int kBfly = 4, kTw = 4;
    static constexpr int kLogTab = kP64LogHmax;
    static constexpr uint32_t kT1 = kP64T1;
    __device__ static constexpr uint32_t t0(uint32_t m) { return p64_t0_offset(m); }
    __device__ __forceinline__ T add(T a, T b) const {
        const T s = a + b;  // < 2p < 2^63
        return s >= kP64 ? s - kP64 : s;
    }
    __device__ __forceinline__ T sub(T a, T b) const { return a >= b ? a - b : a - b + kP64; }
    __device__ __forceinline__ T mulw(T a, W w) const { return mul_mont64(a, w); }
};

__device__ __forceinline__ uint32_t padx(uint32_t i) { return i + (i >> 5); }

// fn(std::integral_constant<int, g>) for every g of the sequence, in order.
template <class Fn, int... G>
__device__ __forceinline__ void for_each_index(Fn &&fn, std::integer_sequence<int, G...>) {
    (fn(std::integral_constant<int, G>{}), ...);
}

template <int R>
__device__ __forceinline__ uint32_t bitrev(uint32_t k) { return __brev(k) >> (32 - R); }

// 2^R-point DIF network on x[base .. base + 2^R): stage t pairs (k, k + h),
// h = 2^(R-t-1), twiddle w_{2^R}^((k mod h) 2^t); w_{2^R} = table[2^kLogTab / 2^R].
template <int R, class F>
__device__ __forceinline__ void small_dif(typename F::T *x, const typename F::W *__restrict__ tw, const F &f) {
#pragma unroll
    for (int t = 0; t < R; ++t) {
        const int h = 1 << (R - t - 1);
#pragma unroll
        for (int k = 0; k < (1 << R); ++k) {
            if (k & h) continue;
            const int nb = (k >> (R - t)) * h + (k & (h - 1));  // butterfly number within the stage
            if (F::kBfly && nb > 0 && nb % F::kBfly == 0) __builtin_amdgcn_sched_barrier(0);
            const int j = (k & (h - 1)) << t;  // exponent of the 2^R-th root
            const typename F::T u = x[k], v = x[k + h];
            x[k] = f.add(u, v);
            const typename F::T d = f.sub(u, v);
            x[k + h] = j == 0 ? d : f.mulw(d, tw[j * ((1u << F::kLogTab) >> R)]);
        }
        __builtin_amdgcn_sched_barrier(0);  // one stage at a time: bounds live registers
    }
}

// Inverse of small_dif up to the factor 2^R: stages in reverse order,
// (a, b) -> (a + b w^-j, a - b w^-j).
template <int R, class F>
__device__ __forceinline__ void small_dit_inv(typename F::T *x, const typename F::W *__restrict__ itw, const F &f) {
#pragma unroll
    for (int t = R - 1; t >= 0; --t) {
        const int h = 1 << (R - t - 1);
#pragma unroll
        for (int k = 0; k < (1 << R); ++k) {
            if (k & h) continue;
            const int nb = (k >> (R - t)) * h + (k & (h - 1));  // butterfly number within the stage
            if (F::kBfly && nb > 0 && nb % F::kBfly == 0) __builtin_amdgcn_sched_barrier(0);
            const int j = (k & (h - 1)) << t;
            const typename F::T a = x[k];
            typename F::T b = x[k + h];
            if (j != 0) b = f.mulw(b, itw[j * ((1u << F::kLogTab) >> R)]);
            x[k] = f.add(a, b);
            x[k + h] = f.sub(a, b);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Position k of a group with offset lo in a pass starting at stage s gets the
// factor w_L^(2^s lo bitrev_R(k)).  The tables hold these products indexed by
// (bitrev_R(k), lo) with lo fastest, so the lanes of a wave (consecutive lo)
// read consecutive entries: row stride 1024 for pass 0 (lo = gidx < 1024),
// 32 for pass 1 (lo < 32, where w_L^(2^s) = w_1024).
template <int M, int R, uint32_t STRIDE, class F>
__device__ __forceinline__ void twiddle_group(typename F::T *x, const typename F::W *__restrict__ tbl, uint32_t lo,
                                              const F &f) {
#pragma unroll
    for (int k = 1; k < (1 << R); ++k) {
        x[k] = f.mulw(x[k], tbl[STRIDE * bitrev<R>(k) + lo]);
        // Bound the twiddle loads in flight: 8 when registers allow, 4 for the
        // 1024-thread transform (or the field's own bound).
        constexpr int G = F::kTw ? F::kTw : (M >= 15 ? 4 : 8);
        if ((k & (G - 1)) == G - 1) __builtin_amdgcn_sched_barrier(0);
    }
}

// LDS layout: element i of the transform vector lives at word padx(i) =
// i + i/32.  For the three element sets a thread touches the addresses are a
// per-thread base plus a compile-time multiple of k:
//   pass 0  (k 2^10 + gidx, gidx < 2^10):       padx(gidx) + 1056 k
//   pass 1  (hi 2^10 + 32 k + lo, lo < 32):     33 hi + 1024 hi + lo + 33 k
//   pass 2  (32 t + k, k < 32):                 33 t + k
__device__ __forceinline__ uint32_t base_pass1(uint32_t t) {
    const uint32_t lo = t & 31u, hi = t >> 5;
    return (hi << 10) + (hi << 5) + lo;
}

// Forward transform of the 16-bit coefficients of `src` (n32 limbs, zero
// beyond them up to 2^M coefficients); with TW each is first multiplied by
// twist[(i 2^(kLogTab - M)) & tmask] (tmask 0 selects twist[0], which holds
// 1, so both halves of a product run the same branch-free code).  On return
// x[k] holds position 32 t + k of the bit-reversed-order transform.
template <int M, class F, bool TW = false>
__device__ __forceinline__ void ntt_forward(const uint32_t *__restrict__ src, uint32_t n32, typename F::T (&x)[E],
                                            typename F::T *sh, const typename F::W *__restrict__ fw, const F &f,
                                            const typename F::W *__restrict__ twist = nullptr, uint32_t tmask = 0) {
    constexpr int R0 = M - 10;
    constexpr int G0 = E >> R0;
    constexpr uint32_t T = (1u << M) / E;
    const uint32_t t = threadIdx.x;
    // Stage the limbs (zero-padded to L/2 words = L coefficients) in LDS.
    __syncthreads();  // the previous user of sh is done
    uint32_t *sw = reinterpret_cast<uint32_t *>(sh);
    for (uint32_t w = t; w < (1u << M) / 2; w += T) sw[w] = w < n32 ? src[w] : 0u;
    __syncthreads();
    const uint16_t *coef = reinterpret_cast<const uint16_t *>(sh);
    // pass 0: stages [0, R0); group g: elements k 2^10 + gidx, gidx = t + T g
#pragma unroll
    for (int g = 0; g < G0; ++g) {
        const uint32_t gidx = t + T * g;
#pragma unroll
        for (int k = 0; k < (1 << R0); ++k) {
            const uint32_t i = gidx + (uint32_t(k) << 10);
            x[g * (1 << R0) + k] = coef[i];
            if constexpr (TW)
                x[g * (1 << R0) + k] = f.mulw(x[g * (1 << R0) + k], twist[(i << (F::kLogTab - M)) & tmask]);
            if (F::kTw && (k & (F::kTw - 1)) == F::kTw - 1) __builtin_amdgcn_sched_barrier(0);
        }
    }
    __syncthreads();  // staging is overwritten below
#pragma unroll
    for (int g = 0; g < G0; ++g) {
        const uint32_t gidx = t + T * g;
        small_dif<R0>(x + g * (1 << R0), fw, f);
        twiddle_group<M, R0, 1024>(x + g * (1 << R0), fw + F::t0(M), gidx, f);
        typename F::T *q = sh + padx(gidx);
#pragma unroll
        for (int k = 0; k < (1 << R0); ++k) q[1056 * k] = x[g * (1 << R0) + k];
    }
    __syncthreads();
    // pass 1: stages [R0, R0 + 5); lo = t mod 32, hi = t / 32
    {
        typename F::T *q = sh + base_pass1(t);
#pragma unroll
        for (int k = 0; k < 32; ++k) x[k] = q[33 * k];
        small_dif<5>(x, fw, f);
        twiddle_group<M, 5, 32>(x, fw + F::kT1, t & 31u, f);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 32; ++k) q[33 * k] = x[k];
        __syncthreads();
    }
    // pass 2: stages [R0 + 5, M); groups are the contiguous runs 32 t .. 32 t + 31
    {
        const typename F::T *q = sh + 33 * t;
#pragma unroll
        for (int k = 0; k < 32; ++k) x[k] = q[k];
        small_dif<5>(x, fw, f);
    }
}

// Inverse of ntt_forward applied to x (position 32 t + k), times `scale`
// (L^-1 times the Montgomery radix) and, with TW, times
// untwist[(i 2^(kLogTab - M)) & tmask] at natural position i; the results for
// i < nout go to dst[i].
template <int M, class F, bool TW = false>
__device__ __forceinline__ void ntt_inverse(typename F::T (&x)[E], typename F::T *__restrict__ dst, uint32_t nout,
                                            typename F::T *sh, const typename F::W *__restrict__ iw, const F &f,
                                            typename F::W scale, const typename F::W *__restrict__ untwist = nullptr,
                                            uint32_t tmask = 0) {
    constexpr int R0 = M - 10;
    constexpr int G0 = E >> R0;
    constexpr uint32_t T = (1u << M) / E;
    const uint32_t t = threadIdx.x;
    small_dit_inv<5>(x, iw, f);
    __syncthreads();
    {
        typename F::T *q = sh + 33 * t;
#pragma unroll
        for (int k = 0; k < 32; ++k) q[k] = x[k];
    }
    __syncthreads();
    {
        typename F::T *q = sh + base_pass1(t);
#pragma unroll
        for (int k = 0; k < 32; ++k) x[k] = q[33 * k];
        twiddle_group<M, 5, 32>(x, iw + F::kT1, t & 31u, f);
        small_dit_inv<5>(x, iw, f);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 32; ++k) q[33 * k] = x[k];
        __syncthreads();
    }
    // one group per element of the index sequence: a compile-time group
    // offset keeps x in registers (a counted loop over 64-bit groups is too
    // large for the unroller and would leave x in scratch memory)
    auto group = [&](auto gc) {
        constexpr int g = decltype(gc)::value;
        const uint32_t gidx = t + T * g;
        typename F::T *y = x + g * (1 << R0);
        const typename F::T *q = sh + padx(gidx);
#pragma unroll
        for (int k = 0; k < (1 << R0); ++k) y[k] = q[1056 * k];
        twiddle_group<M, R0, 1024>(y, iw + F::t0(M), gidx, f);
        small_dit_inv<R0>(y, iw, f);
#pragma unroll
        for (int k = 0; k < (1 << R0); ++k) {
            y[k] = f.mulw(y[k], scale);
            if constexpr (TW) y[k] = f.mulw(y[k], untwist[((gidx + (uint32_t(k) << 10)) << (F::kLogTab - M)) & tmask]);
            if (F::kTw && (k & (F::kTw - 1)) == F::kTw - 1) __builtin_amdgcn_sched_barrier(0);
        }
    };
    for_each_index(group, std::make_integer_sequence<int, G0>{});
    __syncthreads();
    // natural order, unpadded, then contiguous copy-out
#pragma unroll
    for (int g = 0; g < G0; ++g) {
        const uint32_t gidx = t + T * g;
#pragma unroll
        for (int k = 0; k < (1 << R0); ++k) sh[gidx + (uint32_t(k) << 10)] = x[g * (1 << R0) + k];
    }
    __syncthreads();
    for (uint32_t i = t; i < nout; i += T) dst[i] = sh[i];
}

}  // namespace

// Instances [base, base + chunk) of src, fewer when its count is smaller
// (the count of a ragged class list is read on the device).
template <class Src>
__device__ __forceinline__ uint64_t chunk_count(const Src &src, uint64_t base, uint64_t chunk) {
    const uint64_t c = src.count();
    return c > base ? min(c - base, chunk) : 0;
}

// One workgroup per (instance, operand, prime): the forward transform, stored
// in bit-reversed order to tr[work * L ...] (thread t owns positions
// 32 t .. 32 t + 31), work = 4 (instance - base) + 2 operand + prime.
template <int M, class Src>
__global__ __launch_bounds__((1 << M) / E) void ntt_fwd_kernel(NttConst K, Src src, uint64_t base, uint64_t chunk,
                                                               uint32_t *__restrict__ tr) {
    extern __shared__ __align__(16) uint32_t sh[];
    constexpr uint32_t L = 1u << M;
    const uint64_t cnt = chunk_count(src, base, chunk);
    for (uint64_t work = blockIdx.x; work < 4 * cnt; work += gridDim.x) {
        const InstRef in = src.get(base + (work >> 2));
        const int pr = int(work & 1), op = int((work >> 1) & 1);
        uint32_t x[E];
        ntt_forward<M>(op ? in.b : in.a, in.n, x, sh, K.fwd[pr], Fp32{K.p[pr]});
        uint4 *dst = reinterpret_cast<uint4 *>(tr + work * L + E * threadIdx.x);
#pragma unroll
        for (int q = 0; q < E / 4; ++q) dst[q] = make_uint4(x[4 * q], x[4 * q + 1], x[4 * q + 2], x[4 * q + 3]);
        __syncthreads();
    }
}

// One workgroup per (instance, prime): pointwise product of the two
// transforms, inverse transform, scaling; the coefficient residues overwrite
// the first operand's transform.
template <int M, class Src>
__global__ __launch_bounds__((1 << M) / E) void ntt_inv_kernel(NttConst K, Src src, uint64_t base, uint64_t chunk,
                                                               uint32_t *__restrict__ tr) {
    extern __shared__ __align__(16) uint32_t sh[];
    constexpr uint32_t L = 1u << M;
    const uint64_t cnt = chunk_count(src, base, chunk);
    for (uint64_t work = blockIdx.x; work < 2 * cnt; work += gridDim.x) {
        const uint64_t q2 = work >> 1;
        const uint32_t nout = 4 * src.get(base + q2).n;  // coefficients of the product (the last is 0)
        const int pr = int(work & 1);
        const uint32_t p = K.p[pr], pneg = K.pneg[pr];
        uint32_t *ta = tr + (4 * q2 + pr) * L;        // operand a, prime pr
        const uint32_t *tb = ta + 2 * L;              // operand b, prime pr
        uint32_t x[E];
        const uint4 *va = reinterpret_cast<const uint4 *>(ta + E * threadIdx.x);
        const uint4 *vb = reinterpret_cast<const uint4 *>(tb + E * threadIdx.x);
#pragma unroll
        for (int q = 0; q < E / 4; ++q) {
            const uint4 u = va[q], v = vb[q];
            x[4 * q] = mul_mont(u.x, v.x, p, pneg);
            x[4 * q + 1] = mul_mont(u.y, v.y, p, pneg);
            x[4 * q + 2] = mul_mont(u.z, v.z, p, pneg);
            x[4 * q + 3] = mul_mont(u.w, v.w, p, pneg);
        }
        __syncthreads();  // every thread has read its part of ta before residues overwrite it
        ntt_inverse<M>(x, ta, nout, sh, K.inv[pr], Fp32{p}, make_uint2(K.scale[pr][M], K.scale_sh[pr][M]));
        __syncthreads();
    }
}

// The inverse split in two halves, one workgroup per (instance, prime, half)
// with half the threads of ntt_inv_kernel: the forward transform's positions
// [h L/2, (h+1) L/2) hold the even (h = 0) or odd (h = 1) frequencies in
// bit-reversed order, so each half's pointwise product and inverse of length
// L/2 gives z_h; the coefficients are c_j = z_0[j] + w_L^-j z_1[j] and
// c_{j+L/2} = z_0[j] - w_L^-j z_1[j] (CrtCoefSplit).  Used when the
// full-length inverses are too few to fill the GPU.  z_h overwrites the
// first operand's transform at [h L/2, (h+1) L/2).
template <int M, class Src>
__global__ __launch_bounds__((1 << M) / (2 * E)) void ntt_inv_half_kernel(NttConst K, Src src, uint64_t base,
                                                                          uint64_t chunk, uint32_t *__restrict__ tr) {
    extern __shared__ __align__(16) uint32_t sh[];
    constexpr uint32_t L = 1u << M;
    if constexpr (M > kNttLogLmin) {  // halves need transforms of at least 2^kNttLogLmin points
    const uint64_t cnt = chunk_count(src, base, chunk);
    for (uint64_t work = blockIdx.x; work < 4 * cnt; work += gridDim.x) {
        const uint64_t q2 = work >> 2;
        const int pr = int(work & 1), h = int((work >> 1) & 1);
        const uint32_t p = K.p[pr], pneg = K.pneg[pr];
        uint32_t *ta = tr + (4 * q2 + pr) * L + h * (L / 2);  // operand a, prime pr, this half
        const uint32_t *tb = ta + 2 * L;                      // operand b, prime pr, this half
        uint32_t x[E];
        const uint4 *va = reinterpret_cast<const uint4 *>(ta + E * threadIdx.x);
        const uint4 *vb = reinterpret_cast<const uint4 *>(tb + E * threadIdx.x);
#pragma unroll
        for (int q = 0; q < E / 4; ++q) {
            const uint4 u = va[q], v = vb[q];
            x[4 * q] = mul_mont(u.x, v.x, p, pneg);
            x[4 * q + 1] = mul_mont(u.y, v.y, p, pneg);
            x[4 * q + 2] = mul_mont(u.z, v.z, p, pneg);
            x[4 * q + 3] = mul_mont(u.w, v.w, p, pneg);
        }
        __syncthreads();  // every thread has read its part of ta before results overwrite it
        // scale by the full length's L^-1 2^32: z_h then combine without a factor 1/2
        ntt_inverse<M - 1>(x, ta, L / 2, sh, K.inv[pr], Fp32{p}, make_uint2(K.scale[pr][M], K.scale_sh[pr][M]));
        __syncthreads();
    }
    }
}

// Product coefficient k (16-bit position) of chunk slot q from the two
// residues (Garner): residues of prime i at tr + (4 q + i) L.
struct CrtCoef {
    const uint32_t *tr;
    uint32_t L, p1, p2, crt, crt_sh;
    __device__ __forceinline__ uint64_t from(uint32_t a1, uint32_t a2) const {
        const uint32_t tq = mul_shoup(sub_mod(a2, a1, p2), crt, crt_sh, p2);
        return uint64_t(p1) * tq + a1;  // < p1 p2; equals the coefficient (< 2^46)
    }
    __device__ __forceinline__ uint64_t operator()(uint64_t q, uint32_t k) const {
        return from(tr[4 * q * L + k], tr[(4 * q + 1) * L + k]);
    }
    // coefficients k0 .. k0 + 7 (k0 a multiple of 8, k0 + 7 < L), vector loads
    __device__ __forceinline__ void eight(uint64_t q, uint32_t k0, uint64_t (&c)[8]) const {
        const uint4 *r1 = reinterpret_cast<const uint4 *>(tr + 4 * q * L + k0);
        const uint4 *r2 = reinterpret_cast<const uint4 *>(tr + (4 * q + 1) * L + k0);
        const uint4 x0 = r1[0], x1 = r1[1], y0 = r2[0], y1 = r2[1];
        c[0] = from(x0.x, y0.x); c[1] = from(x0.y, y0.y); c[2] = from(x0.z, y0.z); c[3] = from(x0.w, y0.w);
        c[4] = from(x1.x, y1.x); c[5] = from(x1.y, y1.y); c[6] = from(x1.z, y1.z); c[7] = from(x1.w, y1.w);
    }
};

// The same from the two inverse halves of ntt_inv_half_kernel: residue of
// prime i at position k is z_0[j] +- w_L^-j z_1[j] (j = k mod L/2, minus for
// k >= L/2), with z_h at tr + (4 q + i) L + h L/2.
struct CrtCoefSplit {
    const uint32_t *tr;
    const uint2 *inv[kNttPrimes];  // w^-e tables, w of order 2^kNttLogLmax
    uint32_t L, shift, p1, p2, crt, crt_sh;  // shift = kNttLogLmax - log2 L
    __device__ __forceinline__ uint32_t residue(uint64_t q, int i, uint32_t k, uint32_t p) const {
        const uint32_t half = L / 2, j = k & (half - 1);
        const uint32_t *z = tr + (4 * q + i) * L;
        const uint2 w = inv[i][j << shift];
        const uint32_t t = mul_shoup(z[half + j], w.x, w.y, p);
        return k < half ? add_mod(z[j], t, p) : sub_mod(z[j], t, p);
    }
    __device__ __forceinline__ uint64_t operator()(uint64_t q, uint32_t k) const {
        const uint32_t a1 = residue(q, 0, k, p1), a2 = residue(q, 1, k, p2);
        const uint32_t tq = mul_shoup(sub_mod(a2, a1, p2), crt, crt_sh, p2);
        return uint64_t(p1) * tq + a1;
    }
    // residues k0 .. k0 + 7 of prime i (k0 a multiple of 8): z words and,
    // at full table resolution (shift 0), the twiddles by vector loads
    __device__ __forceinline__ void residue8(uint64_t q, int i, uint32_t k0, uint32_t p, uint32_t (&r)[8]) const {
        const uint32_t half = L / 2, j0 = k0 & (half - 1);
        const uint32_t *z = tr + (4 * q + i) * L;
        const uint4 *z0 = reinterpret_cast<const uint4 *>(z + j0), *z1 = reinterpret_cast<const uint4 *>(z + half + j0);
        const uint4 a0 = z0[0], a1 = z0[1], b0 = z1[0], b1 = z1[1];
        const uint32_t av[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
        const uint32_t bv[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
        uint2 w[8];
        if (shift == 0) {
            const uint4 *wt = reinterpret_cast<const uint4 *>(inv[i] + j0);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint4 t = wt[e];
                w[2 * e] = make_uint2(t.x, t.y);
                w[2 * e + 1] = make_uint2(t.z, t.w);
            }
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) w[e] = inv[i][(j0 + e) << shift];
        }
        const bool lo = k0 < half;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const uint32_t t = mul_shoup(bv[e], w[e].x, w[e].y, p);
            r[e] = lo ? add_mod(av[e], t, p) : sub_mod(av[e], t, p);
        }
    }
    __device__ __forceinline__ void eight(uint64_t q, uint32_t k0, uint64_t (&c)[8]) const {
        uint32_t a1[8], a2[8];
        residue8(q, 0, k0, p1, a1);
        residue8(q, 1, k0, p2, a2);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const uint32_t tq = mul_shoup(sub_mod(a2[e], a1[e], p2), crt, crt_sh, p2);
            c[e] = uint64_t(p1) * tq + a1[e];
        }
    }
};

// Product coefficient k from the PrimeField64 half results: cyclic at
// tr + 4 q H, negacyclic at tr + (4 q + 1) H.  c_lo = (cyc + neg) / 2 and
// c_hi = (cyc - neg) / 2, each below 2^46 < p, so the sum (difference) mod p
// is twice the coefficient exactly.
struct Half64Coef {
    const uint64_t *tr;
    uint32_t H;
    __device__ __forceinline__ uint64_t operator()(uint64_t q, uint32_t k) const {
        const uint64_t *cyc = tr + 4 * q * H, *neg = cyc + H;
        const uint32_t j = k < H ? k : k - H;
        const uint64_t c = cyc[j], n = neg[j];
        uint64_t v;
        if (k < H) {
            v = c + n;
            if (v >= kP64) v -= kP64;
        } else {
            v = c >= n ? c - n : c - n + kP64;
        }
        return v >> 1;
    }
    __device__ __forceinline__ void eight(uint64_t q, uint32_t k0, uint64_t (&c)[8]) const {
        const uint64_t *cyc = tr + 4 * q * H, *neg = cyc + H;
        const bool lo = k0 < H;
        const uint32_t j0 = lo ? k0 : k0 - H;
        const ulonglong2 *cv = reinterpret_cast<const ulonglong2 *>(cyc + j0);
        const ulonglong2 *nv = reinterpret_cast<const ulonglong2 *>(neg + j0);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const ulonglong2 cc = cv[e], nn = nv[e];
            const uint64_t cs[2] = {cc.x, cc.y}, ns[2] = {nn.x, nn.y};
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                uint64_t v;
                if (lo) {
                    v = cs[h] + ns[h];
                    if (v >= kP64) v -= kP64;
                } else {
                    v = cs[h] >= ns[h] ? cs[h] - ns[h] : cs[h] - ns[h] + kP64;
                }
                c[2 * e + h] = v >> 1;
            }
        }
    }
};

// One workgroup per instance: coefficients from `coef`, per-thread combine of
// 8 coefficients into 4 low words and 2 high words, L + H.
template <int NW, class Src, class Coef>
__global__ __launch_bounds__(64 * NW) void ntt_crt_carry_kernel(Coef coef, Src src, uint64_t base, uint64_t chunk) {
    extern __shared__ __align__(16) uint32_t lds[];
    const uint64_t cnt = chunk_count(src, base, chunk);
    for (uint64_t q = blockIdx.x; q < cnt; q += gridDim.x) {
        const InstRef in = src.get(base + q);
        const uint32_t nout = 4 * in.n;
        const uint32_t nwords = 2 * in.n;
        const uint32_t ngroups = (nwords + 3) / 4;
        uint32_t *Lsh = lds;                                          // [4 ngroups]
        uint2 *Hsh = reinterpret_cast<uint2 *>(Lsh + 4 * ngroups);    // [ngroups]
        uint32_t *summary = reinterpret_cast<uint32_t *>(Hsh + ngroups);
        for (uint32_t g = threadIdx.x; g < ngroups; g += 64 * NW) {
            // column sums of sum_e c_{8g+e} 2^(16 e), one 64-bit column per word
            uint64_t col[6] = {0, 0, 0, 0, 0, 0};
            uint64_t cf[8];
            coef.eight(q, 8 * g, cf);  // 8 g + 7 < L (the padded length is a multiple of 8)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const uint32_t k = 8 * g + e;
                const uint64_t c = k < nout ? cf[e] : 0;
                const uint64_t v = c << (16 * (e & 1));  // < 2^62
                col[e >> 1] += uint32_t(v);
                col[(e >> 1) + 1] += uint32_t(v >> 32);
            }
            uint64_t carry = 0;
            uint32_t R[6];
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                const uint64_t sv = col[j] + carry;
                R[j] = uint32_t(sv);
                carry = sv >> 32;
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) Lsh[4 * g + j] = R[j];
            Hsh[g] = make_uint2(R[4], R[5]);
        }
        __syncthreads();
        wg_add_rows<NW>(LHSrc4{Lsh, Hsh, nwords}, in.c, nwords, summary);
        __syncthreads();
    }
}

// Coefficients to words, one thread per group of 8 coefficients (16-bit
// positions) over all instances of the round: their column sums are folded
// into 4 low words L[4 g ..] and a high pair H[g] (positions 4 g + 4, 4 g + 5)
// in the instance's word area lh + q * lh_stride (L, then H at 4 gmax).
template <class Src, class Coef>
__global__ __launch_bounds__(256) void ntt_fold_kernel(Coef coef, Src src, uint64_t base, uint64_t chunk,
                                                       uint32_t *__restrict__ lh, uint64_t lh_stride, uint32_t gmax) {
    const uint64_t cnt = chunk_count(src, base, chunk);
    for (uint64_t item = uint64_t(blockIdx.x) * 256 + threadIdx.x; item < cnt * gmax;
         item += uint64_t(gridDim.x) * 256) {
        const uint64_t q = item / gmax;
        const uint32_t g = uint32_t(item - q * gmax);
        const uint32_t n = src.get(base + q).n;
        const uint32_t nout = 4 * n, ngroups = (2 * n + 3) / 4;
        if (g >= ngroups) continue;
        // column sums of sum_e c_{8g+e} 2^(16 e), one 64-bit column per word
        uint64_t col[6] = {0, 0, 0, 0, 0, 0};
        uint64_t cf[8];
        coef.eight(q, 8 * g, cf);  // 8 g + 7 < L (the padded length is a multiple of 8)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const uint32_t k = 8 * g + e;
            const uint64_t c = k < nout ? cf[e] : 0;
            const uint64_t v = c << (16 * (e & 1));  // < 2^62
            col[e >> 1] += uint32_t(v);
            col[(e >> 1) + 1] += uint32_t(v >> 32);
        }
        uint64_t carry = 0;
        uint32_t R[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            const uint64_t sv = col[j] + carry;
            R[j] = uint32_t(sv);
            carry = sv >> 32;
        }
        uint32_t *L = lh + q * lh_stride;
        *reinterpret_cast<uint4 *>(L + 4 * g) = make_uint4(R[0], R[1], R[2], R[3]);
        reinterpret_cast<uint2 *>(L + 4 * gmax)[g] = make_uint2(R[4], R[5]);
    }
}

// One workgroup per instance: the product = L + H with the ballot-adder,
// the addends of all R rows of a wave read at once into registers (chunk c:
// L words 4 c .. 4 c + 3 and H's pair c - 1 at words 4 c, 4 c + 1).
template <int NW, int R, class Src>
__global__ __launch_bounds__(64 * NW) void ntt_carry_kernel(Src src, uint64_t base, uint64_t chunk,
                                                            const uint32_t *__restrict__ lh, uint64_t lh_stride,
                                                            uint32_t gmax) {
    __shared__ uint32_t summary[NW];
    const uint64_t cnt = chunk_count(src, base, chunk);
    const uint32_t lane = lane_id(), w = wave_in_block();
    for (uint64_t q = blockIdx.x; q < cnt; q += gridDim.x) {
        const InstRef in = src.get(base + q);
        const uint32_t nwords = 2 * in.n, nchunks = (nwords + 3) / 4;
        const uint32_t *L = lh + q * lh_stride;
        const uint2 *H = reinterpret_cast<const uint2 *>(L + 4 * gmax);
        uint32_t x[R][4], y[R][4];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const uint32_t c = 64 * (w * uint32_t(R) + uint32_t(i)) + lane;
            const bool in_l = c < nchunks, in_h = in_l && c >= 1;
            const uint4 l = reinterpret_cast<const uint4 *>(L)[in_l ? c : 0u];
            const uint2 h = H[in_h ? c - 1 : 0u];
            x[i][0] = l.x; x[i][1] = l.y; x[i][2] = l.z; x[i][3] = l.w;
            y[i][0] = in_h ? h.x : 0u;
            y[i][1] = in_h ? h.y : 0u;
            y[i][2] = y[i][3] = 0u;
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (!in_l || 4 * c + uint32_t(t) >= nwords) x[i][t] = y[i][t] = 0u;
        }
        const GlobalSink sink{in.c, nwords, (reinterpret_cast<uintptr_t>(in.c) & 15) == 0};
        (void)wg_add_regs<NW, R>(x, y, nwords, sink, summary);
        __syncthreads();  // summary is free for the next instance
    }
}

// PrimeField64, one workgroup per (instance, operand, half): the forward
// transform of length H = 2^M of the operand (half 1: twisted by psi^i), in
// bit-reversed order to tr[work * H ...], work = 4 (instance - base) + 2
// operand + half.
template <int M, class Src>
__global__ __launch_bounds__((1 << M) / E) void ntt64_fwd_kernel(NttConst64 K, Src src, uint64_t base, uint64_t chunk,
                                                                 uint64_t *__restrict__ tr) {
    extern __shared__ __align__(16) uint64_t sh64[];
    constexpr uint32_t H = 1u << M;
    const uint64_t cnt = chunk_count(src, base, chunk);
    for (uint64_t work = blockIdx.x; work < 4 * cnt; work += gridDim.x) {
        const InstRef in = src.get(base + (work >> 2));
        const int half = int(work & 1), op = int((work >> 1) & 1);
        uint64_t x[E];
        ntt_forward<M, Fp64, true>(op ? in.b : in.a, in.n, x, sh64, K.fwd, Fp64{}, K.twist, half ? ~0u : 0u);
        ulonglong2 *dst = reinterpret_cast<ulonglong2 *>(tr + work * H + E * threadIdx.x);
#pragma unroll
        for (int q = 0; q < E / 2; ++q) dst[q] = make_ulonglong2(x[2 * q], x[2 * q + 1]);
        __syncthreads();
    }
}

// PrimeField64, one workgroup per (instance, half): pointwise Montgomery
// product of the two operands' transforms, inverse transform, scaling (and
// for half 1 the untwist by psi^-i); the H results overwrite operand a's
// transform of that half.
template <int M, class Src>
__global__ __launch_bounds__((1 << M) / E) void ntt64_inv_kernel(NttConst64 K, Src src, uint64_t base, uint64_t chunk,
                                                                 uint64_t *__restrict__ tr) {
    extern __shared__ __align__(16) uint64_t sh64[];
    constexpr uint32_t H = 1u << M;
    const uint64_t cnt = chunk_count(src, base, chunk);
    for (uint64_t work = blockIdx.x; work < 2 * cnt; work += gridDim.x) {
        const uint64_t q2 = work >> 1;
        const int half = int(work & 1);
        uint64_t *ta = tr + (4 * q2 + half) * H;  // operand a, this half
        const uint64_t *tb = ta + 2 * H;          // operand b, this half
        uint64_t x[E];
        const ulonglong2 *va = reinterpret_cast<const ulonglong2 *>(ta + E * threadIdx.x);
        const ulonglong2 *vb = reinterpret_cast<const ulonglong2 *>(tb + E * threadIdx.x);
#pragma unroll
        for (int q = 0; q < E / 2; ++q) {
            const ulonglong2 u = va[q], v = vb[q];
            x[2 * q] = mul_mont64(u.x, v.x);
            x[2 * q + 1] = mul_mont64(u.y, v.y);
        }
        __syncthreads();  // every thread has read its part of ta before results overwrite it
        ntt_inverse<M, Fp64, true>(x, ta, H, sh64, K.inv, Fp64{}, K.scale[M], K.untwist, half ? ~0u : 0u);
        __syncthreads();
    }
}

template <int NW, class Src, class Coef>
static hipError_t launch_crt_nw(const Coef &coef, const Src &src, uint64_t base, uint64_t chunk, uint64_t grid,
                                uint32_t nmax, hipStream_t st) {
    const uint32_t ngroups = (2 * nmax + 3) / 4;
    const size_t lds = sizeof(uint32_t) * (4 * ngroups + 2 * ngroups + NW);
    static std::atomic<uint64_t> lds_set{0};
    hipError_t e = lds_limit_once(reinterpret_cast<const void *>(&ntt_crt_carry_kernel<NW, Src, Coef>), lds_set);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((ntt_crt_carry_kernel<NW, Src, Coef>), dim3(uint32_t(grid)), dim3(64 * NW), lds, st, coef, src,
                       base, chunk);
    return hipGetLastError();
}

// Coefficients to product for the `chunk`-instance round starting at base;
// `grid` caps the per-instance workgroups.  Up to 8192 output words one
// workgroup per instance recombines, folds into LDS and carries (enough
// instances fill the GPU); above, a wide kernel folds all instances' words
// into lh (each instance's area of 6 gmax words at lh + q lh_stride, the free
// second-operand half of its transform scratch) and a workgroup per instance
// only carries, since few instances of that size would leave CUs idle.
template <class Src, class Coef>
static hipError_t launch_crt(const Coef &coef, const Src &src, uint64_t base, uint64_t chunk, uint64_t grid,
                             uint32_t nmax, uint32_t *lh, uint64_t lh_stride, hipStream_t st) {
    const uint32_t gmax = (2 * nmax + 3) / 4;
    if (gmax <= 256) return launch_crt_nw<4>(coef, src, base, chunk, grid, nmax, st);
    if (gmax <= 1024) return launch_crt_nw<8>(coef, src, base, chunk, grid, nmax, st);
    if (gmax <= 2048) return launch_crt_nw<16>(coef, src, base, chunk, grid, nmax, st);
    const uint64_t items = std::min(chunk, grid * 65536) * gmax;
    hipLaunchKernelGGL((ntt_fold_kernel<Src, Coef>), dim3(uint32_t(std::min<uint64_t>((items + 255) / 256, 65536))),
                       dim3(256), 0, st, coef, src, base, chunk, lh, lh_stride, gmax);
    // 16 waves of 4 rows: up to 16384 words (gmax <= 4096)
    hipLaunchKernelGGL((ntt_carry_kernel<16, 4, Src>), dim3(uint32_t(grid)), dim3(1024), 0, st, src, base, chunk, lh,
                       lh_stride, gmax);
    return hipGetLastError();
}

// The three kernels of a product over instances [0, count_max) of src in
// rounds of `chunk` instances (each round's transforms fill tr).  Grids are
// capped at `cap` workgroups per kernel (the kernels loop over their work).
template <int M, class Src>
static hipError_t launch_ntt_m(const NttConst &K, const Src &src, uint32_t nmax, uint64_t count_max, uint64_t chunk,
                               uint64_t cap, uint32_t *tr, hipStream_t st, int num_cus) {
    const size_t lds = sizeof(uint32_t) * ((1u << M) + (1u << M) / 32);
    const size_t lds_half = sizeof(uint32_t) * ((1u << (M - 1)) + (1u << (M - 1)) / 32);
    static std::atomic<uint64_t> lds_set[3];
    const void *fns[3] = {reinterpret_cast<const void *>(&ntt_fwd_kernel<M, Src>),
                          reinterpret_cast<const void *>(&ntt_inv_kernel<M, Src>),
                          reinterpret_cast<const void *>(&ntt_inv_half_kernel<M, Src>)};
    for (int i = 0; i < 3; ++i) {
        const hipError_t e = lds_limit_once(fns[i], lds_set[i]);
        if (e != hipSuccess) return e;
    }
    const uint32_t T = (1u << M) / E;
    const uint32_t L = 1u << M;
    // workgroups of length 2^M that fit one CU's LDS at once
    const uint64_t per_cu = (160 * 1024) / lds;
    for (uint64_t base = 0; base < count_max; base += chunk) {
        const uint64_t c = std::min(chunk, count_max - base);
        hipLaunchKernelGGL((ntt_fwd_kernel<M, Src>), dim3(uint32_t(std::min(4 * c, cap))), dim3(T), lds, st, K, src, base,
                           chunk, tr);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        // 2c full-length inverses that leave CUs idle: run them as 4c halves
        const bool split = M > kNttLogLmin && 2 * c < per_cu * uint64_t(num_cus > 0 ? num_cus : 1);
        if (split) {
            hipLaunchKernelGGL((ntt_inv_half_kernel<M, Src>), dim3(uint32_t(std::min(4 * c, cap))), dim3(T / 2),
                               lds_half, st, K, src, base, chunk, tr);
        } else {
            hipLaunchKernelGGL((ntt_inv_kernel<M, Src>), dim3(uint32_t(std::min(2 * c, cap))), dim3(T), lds, st, K, src,
                               base, chunk, tr);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        // words go to the second operand's transforms (slots 4 q + 2, 4 q + 3)
        if (split) {
            const CrtCoefSplit coef{tr, {K.inv[0], K.inv[1]}, L, uint32_t(kNttLogLmax - M), K.p[0], K.p[1], K.crt,
                                    K.crt_sh};
            e = launch_crt(coef, src, base, chunk, std::min(c, cap), nmax, tr + 2 * L, 4 * uint64_t(L), st);
        } else {
            const CrtCoef coef{tr, L, K.p[0], K.p[1], K.crt, K.crt_sh};
            e = launch_crt(coef, src, base, chunk, std::min(c, cap), nmax, tr + 2 * L, 4 * uint64_t(L), st);
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <class Src>
static hipError_t launch_ntt(const NttConst &K, const Src &src, uint32_t nmax, uint64_t count_max, uint64_t chunk,
                             uint64_t cap, uint32_t *tr, hipStream_t st, int num_cus) {
    switch (ntt_log_len(nmax)) {
        case 11: return launch_ntt_m<11>(K, src, nmax, count_max, chunk, cap, tr, st, num_cus);
        case 12: return launch_ntt_m<12>(K, src, nmax, count_max, chunk, cap, tr, st, num_cus);
        case 13: return launch_ntt_m<13>(K, src, nmax, count_max, chunk, cap, tr, st, num_cus);
        case 14: return launch_ntt_m<14>(K, src, nmax, count_max, chunk, cap, tr, st, num_cus);
        case 15: return launch_ntt_m<15>(K, src, nmax, count_max, chunk, cap, tr, st, num_cus);
        default: return hipErrorInvalidValue;
    }
}

size_t ntt_list_scratch_bytes(uint64_t count) {
    // at most kNttListChunk instances of the longest transform per round
    const uint64_t c = count < kNttListChunk ? count : kNttListChunk;
    return size_t(c) * 4 * kNttLmax * sizeof(uint32_t);
}

hipError_t launch_bigmul_ntt_list(const NttConst &K, const ListInst &src, uint32_t nmax, uint64_t count_max,
                                  uint32_t *scratch, hipStream_t st, int num_cus) {
    const uint32_t m = ntt_log_len(nmax);
    if (m == 0) return hipErrorInvalidValue;
    if (count_max == 0) return hipSuccess;
    // rounds of as many instances as the scratch holds at this length
    const uint64_t cmax = count_max < kNttListChunk ? count_max : kNttListChunk;
    const uint64_t chunk = cmax << (kNttLogLmax - m);
    // about two resident workgroups per CU (2^(15-M) fit at length 2^M)
    const uint64_t cap = uint64_t(num_cus) << (16 - m);
    return launch_ntt(K, src, nmax, count_max, chunk, cap, scratch, st, num_cus);
}

uint32_t ntt_log_len(uint32_t n32) {
    uint32_t m = 11;  // smallest supported transform (64 threads)
    while ((1u << m) < 4 * n32) ++m;
    return m <= uint32_t(kNttLogLmax) ? m : 0;
}

size_t ntt_scratch_bytes(uint32_t n32, uint64_t batch) {
    const uint32_t m = ntt_log_len(n32);
    return m ? size_t(batch) * 4 * (size_t(1) << m) * sizeof(uint32_t) : 0;
}

hipError_t launch_bigmul_ntt(const NttConst &K, const uint32_t *a, const uint32_t *b, uint32_t *c, uint32_t n32,
                             uint64_t batch, uint32_t *tr, hipStream_t st, uint64_t round, int num_cus) {
    if (batch == 0) return hipSuccess;
    if (round == 0) return hipErrorInvalidValue;
    return launch_ntt(K, UniformInst{a, b, c, n32, batch}, n32, batch, std::min(batch, round), 65536, tr, st,
                      num_cus);
}

// The three PrimeField64 kernels over instances [0, count_max) of src in rounds
// of `chunk` instances; grids capped at `cap` workgroups.
template <int M, class Src>
static hipError_t launch_ntt64_m(const NttConst64 &K, const Src &src, uint32_t nmax, uint64_t count_max,
                                 uint64_t chunk, uint64_t cap, uint64_t *tr, hipStream_t st) {
    const size_t lds = sizeof(uint64_t) * ((1u << M) + (1u << M) / 32);
    const void *fns[2] = {reinterpret_cast<const void *>(&ntt64_fwd_kernel<M, Src>),
                          reinterpret_cast<const void *>(&ntt64_inv_kernel<M, Src>)};
    static std::atomic<uint64_t> lds_set[2];
    for (int i = 0; i < 2; ++i) {
        const hipError_t e = lds_limit_once(fns[i], lds_set[i]);
        if (e != hipSuccess) return e;
    }
    const uint32_t T = (1u << M) / E;
    const Half64Coef coef{tr, 1u << M};
    for (uint64_t base = 0; base < count_max; base += chunk) {
        const uint64_t c = std::min(chunk, count_max - base);
        hipLaunchKernelGGL((ntt64_fwd_kernel<M, Src>), dim3(uint32_t(std::min(4 * c, cap))), dim3(T), lds, st, K, src,
                           base, chunk, tr);
        hipLaunchKernelGGL((ntt64_inv_kernel<M, Src>), dim3(uint32_t(std::min(2 * c, cap))), dim3(T), lds, st, K, src,
                           base, chunk, tr);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        // words go to the second operand's transforms (slots 4 q + 2, 4 q + 3)
        uint32_t *lh = reinterpret_cast<uint32_t *>(tr + 2 * (uint64_t(1) << M));
        e = launch_crt(coef, src, base, chunk, std::min(c, cap), nmax, lh, 8 * (uint64_t(1) << M), st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <class Src>
static hipError_t launch_ntt64(const NttConst64 &K, const Src &src, uint32_t nmax, uint64_t count_max,
                               uint64_t chunk, uint64_t cap, uint64_t *tr, hipStream_t st) {
    switch (ntt64_log_len(nmax)) {
        case 11: return launch_ntt64_m<11>(K, src, nmax, count_max, chunk, cap, tr, st);
        case 12: return launch_ntt64_m<12>(K, src, nmax, count_max, chunk, cap, tr, st);
        case 13: return launch_ntt64_m<13>(K, src, nmax, count_max, chunk, cap, tr, st);
        case 14: return launch_ntt64_m<14>(K, src, nmax, count_max, chunk, cap, tr, st);
        default: return hipErrorInvalidValue;
    }
}

// H covers the 2 n32 coefficients of an operand (the cyclic and negacyclic
// halves together hold the 4 n32 coefficients of the product).
uint32_t ntt64_log_len(uint32_t n32) {
    uint32_t m = kP64LogHmin;
    while ((1u << m) < 2 * n32) ++m;
    return m <= uint32_t(kP64LogHmax) ? m : 0;
}

size_t ntt64_scratch_bytes(uint32_t n32, uint64_t batch) {
    const uint32_t m = ntt64_log_len(n32);
    return m ? size_t(batch) * 4 * (size_t(1) << m) * sizeof(uint64_t) : 0;
}

size_t ntt64_list_scratch_bytes(uint64_t count) {
    const uint64_t c = count < kNttListChunk ? count : kNttListChunk;
    return size_t(c) * 4 * kP64Hmax * sizeof(uint64_t);
}

hipError_t launch_bigmul_ntt64(const NttConst64 &K, const uint32_t *a, const uint32_t *b, uint32_t *c, uint32_t n32,
                               uint64_t batch, uint64_t *tr, hipStream_t st, uint64_t round) {
    if (batch == 0) return hipSuccess;
    if (round == 0) return hipErrorInvalidValue;
    return launch_ntt64(K, UniformInst{a, b, c, n32, batch}, n32, batch, std::min(batch, round), 65536, tr, st);
}

hipError_t launch_bigmul_ntt64_list(const NttConst64 &K, const ListInst &src, uint32_t nmax, uint64_t count_max,
                                    uint64_t *scratch, hipStream_t st, int num_cus) {
    const uint32_t m = ntt64_log_len(nmax);
    if (m == 0) return hipErrorInvalidValue;
    if (count_max == 0) return hipSuccess;
    // rounds of as many instances as the scratch holds at this length
    const uint64_t cmax = count_max < kNttListChunk ? count_max : kNttListChunk;
    const uint64_t chunk = cmax << (kP64LogHmax - m);
    // about two resident workgroups per CU (2^(14-M) fit at length 2^M)
    const uint64_t cap = uint64_t(num_cus) << (15 - m);
    return launch_ntt64(K, src, nmax, count_max, chunk, cap, scratch, st);
}

// ---------------------------------------------------------------------------
// One product beyond 2^18 bits as a two-dimensional convolution.  With the
// operands cut into k blocks of bw words (2 bw 16-bit coefficients each),
//     A(x, y) = sum_q sum_j a_{q,j} x^j y^q   (and B alike),
// the integer product is C(x, y) = A B evaluated at x = 2^16, y = 2^(32 bw).
// Zero-padding x to L >= 4 bw points and y to K = 2H >= 2k - 1 points makes
// both cyclic convolutions exact, so C is the inverse of the pointwise product
// of the two-dimensional transforms: rows (length L, per block, the transform
// kernels above) and columns (length K, across blocks, per row position).
// Each entry c(v, u) is below k 2 bw (2^16 - 1)^2 <= 2^52 < p1 p2, so CRT
// recovers it exactly, and coefficient P of the product is
// c(P div 2bw, P mod 2bw) + c(P div 2bw - 1, P mod 2bw + 2bw).
//
// Transform slots (L words each) in the scratch: forward rows of block q at
// 4 q + 2 operand + prime (as the batched forward kernel writes them); the
// column kernel overwrites them in place with the product rows, row v of
// prime pr at slot 2 v + pr (a thread owns one column of one prime and reads
// all of its entries before writing any).
// ---------------------------------------------------------------------------

// Two waves per (64 columns x, prime): the K-point column transforms of a
// and b as their even (cyclic, H points; wave 0) and odd (negacyclic: inputs
// times psi^i, psi of order K; wave 1) halves, pointwise Montgomery
// products, H-point inverses, then through LDS the recombination
// c_j = (E_j + psi^-j O_j) / K (wave 0), c_{j+H} = (E_j - psi^-j O_j) / K
// (wave 1), and the scale that undoes the Montgomery factor and the row
// transform's L.
template <int R>
__global__ __launch_bounds__(128) void ntt_col_kernel(NttConst K, uint32_t *__restrict__ tr, uint32_t L, uint32_t M,
                                                      uint32_t k) {
    constexpr int H = 1 << R;
    __shared__ uint32_t hsh[2][H * 64];  // E_j and psi^-j O_j of lane l at [64 j + l]
    const uint32_t wgs_per_prime = L / 64;
    const int pr = int(blockIdx.x / wgs_per_prime);  // uniform: twiddles come through scalar loads
    const uint32_t half = wave_in_block(), lane = lane_id();
    const uint32_t x = (blockIdx.x - uint32_t(pr) * wgs_per_prime) * 64 + lane;
    const uint32_t p = K.p[pr], pneg = K.pneg[pr];
    const Fp32 f{p};
    const uint2 *fw = K.fwd[pr], *iw = K.inv[pr];
    const uint32_t *col = tr + x;
    auto ld = [&](uint32_t slot) { return col[uint64_t(slot) * L]; };
    uint32_t ya[H], yb[H];
#pragma unroll
    for (int i = 0; i < H; ++i) {
        ya[i] = uint32_t(i) < k ? ld(4 * i + pr) : 0u;
        yb[i] = uint32_t(i) < k ? ld(4 * i + 2 + pr) : 0u;
    }
    if (half) {  // odd half: inputs twisted by psi^i (psi = w^(2^(14 - R)))
#pragma unroll
        for (int i = 0; i < H; ++i) {
            const uint2 ps = fw[uint32_t(i) << (14 - R)];
            ya[i] = f.mulw(ya[i], ps);
            yb[i] = f.mulw(yb[i], ps);
        }
    }
    small_dif<R>(ya, fw, f);
    small_dif<R>(yb, fw, f);
#pragma unroll
    for (int i = 0; i < H; ++i) ya[i] = mul_mont(ya[i], yb[i], p, pneg);
    small_dit_inv<R>(ya, iw, f);
    if (half) {
#pragma unroll
        for (int j = 0; j < H; ++j) ya[j] = f.mulw(ya[j], iw[uint32_t(j) << (14 - R)]);
    }
#pragma unroll
    for (int j = 0; j < H; ++j) hsh[half][64 * j + lane] = ya[j];
    __syncthreads();
    // recombine and scale by 2^-(R + 1 + M) 2^32; rows v < 2k - 1
    const uint2 sc = make_uint2(K.scale[pr][R + 1 + M], K.scale_sh[pr][R + 1 + M]);
    const uint32_t nrows = 2 * k - 1;
    uint32_t *out = tr + x;
#pragma unroll
    for (int j = 0; j < H; ++j) {
        const uint32_t e = hsh[0][64 * j + lane], o = hsh[1][64 * j + lane];
        const uint32_t v = uint32_t(j) + half * H;
        if (v < nrows) out[uint64_t(2 * v + pr) * L] = f.mulw(half ? f.sub(e, o) : f.add(e, o), sc);
    }
}

// One workgroup per product row (slot 2 v + prime): the inverse row
// transform, in place, natural order out (the column kernel applied every
// scale factor).
template <int M>
__global__ __launch_bounds__((1 << M) / E) void ntt_rowinv_kernel(NttConst K, uint32_t *__restrict__ tr,
                                                                  uint32_t nslots) {
    extern __shared__ __align__(16) uint32_t sh[];
    constexpr uint32_t L = 1u << M;
    for (uint32_t slot = blockIdx.x; slot < nslots; slot += gridDim.x) {
        const int pr = int(slot & 1u);
        uint32_t *row = tr + uint64_t(slot) * L;
        uint32_t x[E];
        const uint4 *v = reinterpret_cast<const uint4 *>(row + E * threadIdx.x);
#pragma unroll
        for (int q = 0; q < E / 4; ++q) {
            const uint4 u = v[q];
            x[4 * q] = u.x;
            x[4 * q + 1] = u.y;
            x[4 * q + 2] = u.z;
            x[4 * q + 3] = u.w;
        }
        __syncthreads();  // every thread has read its part of the row before results overwrite it
        ntt_inverse<M>(x, row, L, sh, K.inv[pr], Fp32{K.p[pr]}, make_uint2(1u, K.one_sh[pr]));
        __syncthreads();
    }
}

// Coefficient P (16-bit position) of the long product from the product rows.
struct LargeCoef {
    const uint32_t *tr;
    uint32_t L, bw2, nrows;  // bw2 = 2 bw coefficients per block; nrows = 2k - 1
    uint32_t p1, p2, crt, crt_sh;
    // Garner: c(v, u) = p1 t + r1 < p1 p2 (it is below 2^52)
    __device__ __forceinline__ uint32_t crt1(uint32_t r1, uint32_t r2) const {
        return mul_shoup(sub_mod(r2, r1, p2), crt, crt_sh, p2);
    }
    // Coefficients P .. P + 3 (P a multiple of 4; bw2 is one too, so they lie
    // in one block row): four rows' reads at once, at clamped rows where a
    // term is absent (the scratch holds 4 k >= 2 nrows + 2 rows).
    __device__ __forceinline__ void four(uint32_t P, uint64_t (&c)[4]) const {
        const uint32_t v = P / bw2, u = P - v * bw2;
        const bool t0 = v < nrows, t1 = v >= 1 && v - 1 < nrows;
        const uint32_t va = t0 ? v : 0u, vb = t1 ? v - 1 : 0u;
        const uint4 a1 = *reinterpret_cast<const uint4 *>(tr + uint64_t(2 * va) * L + u);
        const uint4 a2 = *reinterpret_cast<const uint4 *>(tr + uint64_t(2 * va + 1) * L + u);
        const uint4 b1 = *reinterpret_cast<const uint4 *>(tr + uint64_t(2 * vb) * L + u + bw2);
        const uint4 b2 = *reinterpret_cast<const uint4 *>(tr + uint64_t(2 * vb + 1) * L + u + bw2);
        const uint32_t x1[4] = {a1.x, a1.y, a1.z, a1.w}, x2[4] = {a2.x, a2.y, a2.z, a2.w};
        const uint32_t y1[4] = {b1.x, b1.y, b1.z, b1.w}, y2[4] = {b2.x, b2.y, b2.z, b2.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const uint64_t ca = uint64_t(p1) * crt1(x1[e], x2[e]) + x1[e];
            const uint64_t cb = uint64_t(p1) * crt1(y1[e], y2[e]) + y1[e];
            c[e] = (t0 ? ca : 0ull) + (t1 ? cb : 0ull);  // < 2^53
        }
    }
};

// Coefficients to words: word w of the product is W_w = c(2w) + c(2w+1) 2^16
// < 2^70, written lo_w + m_w 2^32 (m_w < 2^38).  Then
//     product = sum_w S_w 2^(32 w),  S_w = lo_w + (m_{w-1} mod 2^32) + floor(m_{w-2} / 2^32) < 2^34,
// stored as the low words Lw[w] = S_w mod 2^32 and high words Hw[w + 1] =
// floor(S_w / 2^32) for the final addition.  One thread per 8 words w0 ..
// w0 + 7: it reads coefficients 2 w0 - 8 .. 2 w0 + 15 (six groups of four,
// all issued before use) and recomputes the words below its group, so both
// of its output runs, Lw[w0 ..] and Hw[w0 ..], are aligned 8-word stores.
// A workgroup covers one tile of kLargeTileWords words and also records how
// the tile's part of Lw + Hw passes a carry (the status read by
// large_ntt_add_kernel): bit 0 = it carries out by itself, bit 1 = every
// word of its sum is all-ones (it carries out exactly when a carry comes in).
constexpr uint32_t kLargeTileWords = 8 * 256;

// Tile status from the threads' 8-word sums (carry out g, all-ones p), and
// the carry into each thread given the carry cin into the tile.  summary:
// 4 LDS words.  Returns the carry into the calling thread.
__device__ __forceinline__ uint32_t tile_carries(uint32_t g, bool p, uint32_t cin, uint32_t *summary,
                                                 uint8_t *status) {
    const uint32_t lane = lane_id(), w = wave_in_block();
    const uint64_t G = ballot(g != 0), P = ballot(p);
    const WaveCarry w0 = wave_carry(G, P, 0);
    if (lane == 0) summary[w] = w0.out | ((P == ~0ull ? 1u : 0u) << 1);
    __syncthreads();
    uint32_t c = cin, tg = 0, tp = 1;
#pragma unroll
    for (uint32_t v = 0; v < 4; ++v) {
        const uint32_t sv = summary[v];
        if (v < w) c = (sv & 1u) | ((sv >> 1) & c);
        tg = (sv & 1u) | ((sv >> 1) & tg);
        tp &= sv >> 1;
    }
    if (status) *status = uint8_t(tg | (tp << 1));
    __syncthreads();  // summary is free again
    return uint32_t(wave_carry(G, P, c).into >> lane) & 1u;
}

// The 8 words of L + H (carry-in 0) at one thread: carry out and sum.
__device__ __forceinline__ uint32_t fold_sum8(const uint32_t (&lw)[8], const uint32_t (&hw)[8], uint32_t (&sm)[8],
                                              bool &ones) {
    const uint32_t g = add_words<8>(lw, hw, sm);
    ones = all_ones<8>(sm);
    return g;
}

__global__ __launch_bounds__(256) void large_ntt_fold_kernel(LargeCoef coef, uint64_t nwords, uint32_t *__restrict__ Lw,
                                                             uint32_t *__restrict__ Hw, uint8_t *__restrict__ status) {
    __shared__ uint32_t summary[4];
    const uint64_t ngroups = (nwords + 7) / 8, ntiles = (nwords + kLargeTileWords - 1) / kLargeTileWords;
    const uint32_t pmax = uint32_t(2 * nwords - 4);  // last group of four coefficients
    for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint64_t g = tile * 256 + threadIdx.x;
        const bool act = g < ngroups;
        const uint64_t w0 = 8 * g;
        uint64_t cf[24];  // coefficient 2 w0 - 8 + i
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const int64_t P = int64_t(2 * w0) - 8 + 4 * q;
            const bool ok = act && P >= 0 && P <= int64_t(pmax);
            uint64_t c4[4];
            coef.four(ok ? uint32_t(P) : 0u, c4);
#pragma unroll
            for (int e = 0; e < 4; ++e) cf[4 * q + e] = ok ? c4[e] : 0ull;
        }
        // words w0 - 4 + i, i < 12
        uint32_t lo[12];
        uint64_t m[12];
#pragma unroll
        for (int i = 0; i < 12; ++i) {
            const uint64_t c0 = cf[2 * i], c1 = cf[2 * i + 1];
            const uint64_t t = c0 + ((c1 & 0xFFFFu) << 16);  // < 2^53 + 2^32
            lo[i] = uint32_t(t);
            m[i] = (t >> 32) + (c1 >> 16);
        }
        // S_w for w = w0 - 1 + j, j < 9 (i = j + 3)
        uint64_t S[9];
#pragma unroll
        for (int j = 0; j < 9; ++j) S[j] = uint64_t(lo[j + 3]) + uint32_t(m[j + 2]) + (m[j + 1] >> 32);
        uint32_t lw[8], hw[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            lw[j] = uint32_t(S[j + 1]);
            hw[j] = w0 + uint64_t(j) >= 1 ? uint32_t(S[j] >> 32) : 0u;  // Hw[w] = floor(S_(w-1) / 2^32), Hw[0] = 0
        }
        if (act && w0 + 8 <= nwords) {
            uint4 *pl = reinterpret_cast<uint4 *>(Lw + w0), *ph = reinterpret_cast<uint4 *>(Hw + w0);
            pl[0] = make_uint4(lw[0], lw[1], lw[2], lw[3]);
            pl[1] = make_uint4(lw[4], lw[5], lw[6], lw[7]);
            ph[0] = make_uint4(hw[0], hw[1], hw[2], hw[3]);
            ph[1] = make_uint4(hw[4], hw[5], hw[6], hw[7]);
        } else if (act) {
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (w0 + uint64_t(j) < nwords) {
                    Lw[w0 + j] = lw[j];
                    Hw[w0 + j] = hw[j];
                }
        }
        // words at or above nwords are zero (the product has nwords words)
        uint32_t sm[8];
        bool ones = false;
        const uint32_t gc = fold_sum8(lw, hw, sm, ones);
        (void)tile_carries(act ? gc : 0u, act && ones, 0u, summary, threadIdx.x == 0 ? status + tile : nullptr);
    }
}

// product = Lw + Hw (nwords words), one tile per workgroup.  The carry into
// tile t comes from the statuses below it: the nearest tile j < t that does
// not merely propagate gives it (its own carry out), none gives 0.  Every
// read of L, H and the statuses is issued before the scans that use them.
__global__ __launch_bounds__(256) void large_ntt_add_kernel(const uint32_t *__restrict__ Lw,
                                                            const uint32_t *__restrict__ Hw,
                                                            const uint8_t *__restrict__ status, uint32_t *out,
                                                            uint32_t nwords) {
    __shared__ uint32_t summary[4];
    __shared__ uint32_t tile_cin;
    const uint32_t ntiles = (nwords + kLargeTileWords - 1) / kLargeTileWords;
    const uint32_t lane = lane_id(), wave = wave_in_block();
    const GlobalSink sink{out, nwords, (reinterpret_cast<uintptr_t>(out) & 15) == 0};
    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint32_t g = tile * 256 + threadIdx.x, w0 = 8 * g;
        uint32_t lw[8], hw[8];
        if (w0 + 8 <= nwords) {
            const uint4 *pl = reinterpret_cast<const uint4 *>(Lw + w0), *ph = reinterpret_cast<const uint4 *>(Hw + w0);
            const uint4 l0 = pl[0], l1 = pl[1], h0 = ph[0], h1 = ph[1];
            lw[0] = l0.x; lw[1] = l0.y; lw[2] = l0.z; lw[3] = l0.w;
            lw[4] = l1.x; lw[5] = l1.y; lw[6] = l1.z; lw[7] = l1.w;
            hw[0] = h0.x; hw[1] = h0.y; hw[2] = h0.z; hw[3] = h0.w;
            hw[4] = h1.x; hw[5] = h1.y; hw[6] = h1.z; hw[7] = h1.w;
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                lw[j] = w0 + uint32_t(j) < nwords ? Lw[w0 + j] : 0u;
                hw[j] = w0 + uint32_t(j) < nwords ? Hw[w0 + j] : 0u;
            }
        }
        if (wave == 0) {
            // tiles t - 1 - lane - 64 q, nearest first; below tile 0 nothing
            // carries (status 0)
            uint32_t cin = 0;
            for (int64_t base = int64_t(tile) - 1; base >= 0; base -= 64) {
                const int64_t j = base - int64_t(lane);
                const uint32_t sv = j >= 0 ? status[j] : 0u;
                const uint64_t stop = ballot((sv & 2u) == 0);
                if (stop) {
                    cin = __shfl(sv, int(__ffsll(static_cast<unsigned long long>(stop)) - 1)) & 1u;
                    break;
                }
            }
            if (lane == 0) tile_cin = cin;
        }
        uint32_t sm[8];
        bool ones = false;
        const uint32_t gc = fold_sum8(lw, hw, sm, ones);
        __syncthreads();
        const uint32_t c = tile_carries(gc, ones, tile_cin, summary, nullptr);
        add_carry_words<8>(sm, c);
        const uint32_t s0[4] = {sm[0], sm[1], sm[2], sm[3]}, s1[4] = {sm[4], sm[5], sm[6], sm[7]};
        sink(2 * g, s0);
        sink(2 * g + 1, s1);
    }
}

namespace {

struct LargeNttLayout {
    uint32_t k, M, R;
    size_t tr, lw, hw, st, total;
};

LargeNttLayout large_ntt_layout(uint64_t n32, uint32_t bw) {
    LargeNttLayout s;
    s.k = uint32_t((n32 + bw - 1) / bw);
    s.M = ntt_log_len(bw);
    s.R = 0;
    while ((2u << s.R) < 2 * s.k - 1) ++s.R;  // K = 2^(R+1) >= 2k - 1
    const uint64_t nwords = 2 * n32;
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    s.tr = 0;
    s.lw = al(s.tr + size_t(4) * s.k * (size_t(1) << s.M) * sizeof(uint32_t));
    s.hw = al(s.lw + nwords * sizeof(uint32_t));
    s.st = al(s.hw + (nwords + 1) * sizeof(uint32_t));
    s.total = al(s.st + (nwords + kLargeTileWords - 1) / kLargeTileWords);
    return s;
}

template <int M>
hipError_t launch_large_rows(const NttConst &K, const BlockInst &src, uint32_t *tr, uint32_t nslots_inv, bool fwd,
                             hipStream_t st) {
    const size_t lds = sizeof(uint32_t) * ((1u << M) + (1u << M) / 32);
    static std::atomic<uint64_t> lds_set[2];
    const void *fn = fwd ? reinterpret_cast<const void *>(&ntt_fwd_kernel<M, BlockInst>)
                         : reinterpret_cast<const void *>(&ntt_rowinv_kernel<M>);
    hipError_t e = lds_limit_once(fn, lds_set[fwd ? 0 : 1]);
    if (e != hipSuccess) return e;
    const uint32_t T = (1u << M) / E;
    if (fwd)
        hipLaunchKernelGGL((ntt_fwd_kernel<M, BlockInst>), dim3(4 * src.k), dim3(T), lds, st, K, src, 0, src.k, tr);
    else
        hipLaunchKernelGGL((ntt_rowinv_kernel<M>), dim3(nslots_inv), dim3(T), lds, st, K, tr, nslots_inv);
    return hipGetLastError();
}

hipError_t launch_rows(uint32_t M, const NttConst &K, const BlockInst &src, uint32_t *tr, uint32_t nslots_inv, bool fwd,
                       hipStream_t st) {
    switch (M) {
        case 11: return launch_large_rows<11>(K, src, tr, nslots_inv, fwd, st);
        case 12: return launch_large_rows<12>(K, src, tr, nslots_inv, fwd, st);
        case 13: return launch_large_rows<13>(K, src, tr, nslots_inv, fwd, st);
        case 14: return launch_large_rows<14>(K, src, tr, nslots_inv, fwd, st);
        case 15: return launch_large_rows<15>(K, src, tr, nslots_inv, fwd, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_cols(uint32_t R, const NttConst &K, uint32_t *tr, uint32_t M, uint32_t k, hipStream_t st) {
    const uint32_t L = 1u << M;
    const dim3 grid(2 * L / 64), blk(128);
    switch (R) {
        case 0: hipLaunchKernelGGL((ntt_col_kernel<0>), grid, blk, 0, st, K, tr, L, M, k); break;
        case 1: hipLaunchKernelGGL((ntt_col_kernel<1>), grid, blk, 0, st, K, tr, L, M, k); break;
        case 2: hipLaunchKernelGGL((ntt_col_kernel<2>), grid, blk, 0, st, K, tr, L, M, k); break;
        case 3: hipLaunchKernelGGL((ntt_col_kernel<3>), grid, blk, 0, st, K, tr, L, M, k); break;
        case 4: hipLaunchKernelGGL((ntt_col_kernel<4>), grid, blk, 0, st, K, tr, L, M, k); break;
        case 5: hipLaunchKernelGGL((ntt_col_kernel<5>), grid, blk, 0, st, K, tr, L, M, k); break;
        case 6: hipLaunchKernelGGL((ntt_col_kernel<6>), grid, blk, 0, st, K, tr, L, M, k); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

// Blocks of 2^(11..13) words: the smallest that gives at most 32 blocks (64
// at 8192 words).  Measured on one product each (MI355X): 2^19 / 2^20 bits
// fastest with 2048-word blocks (58 / 66 us against 76 / 103 with 512-word
// ones), 2^22 bits with 4096 (104 against 120 with 2048 and 111 with 8192).
uint32_t large_ntt_auto_block(uint64_t n32) {
    uint32_t bw = 2048;
    while (bw < kMaxLimbs32 && (n32 + bw - 1) / bw > kLargeNttMaxBlocks / 2) bw *= 2;
    return bw;
}

size_t large_ntt_scratch_bytes(uint64_t n32, uint32_t bw) { return large_ntt_layout(n32, bw).total; }

hipError_t launch_bigmul_large_ntt(const Ctx &c, const uint32_t *a, const uint32_t *b, uint32_t *out, uint64_t n32,
                                   uint32_t bw, uint8_t *scratch, hipStream_t st) {
    const LargeNttLayout s = large_ntt_layout(n32, bw);
    if (s.M == 0 || s.k == 0 || s.k > kLargeNttMaxBlocks) return hipErrorInvalidValue;
    const NttConst &K = c.ntt.c;
    auto *tr = reinterpret_cast<uint32_t *>(scratch + s.tr);
    auto *Lw = reinterpret_cast<uint32_t *>(scratch + s.lw);
    auto *Hw = reinterpret_cast<uint32_t *>(scratch + s.hw);
    const BlockInst src{a, b, n32, bw, s.k};
    const uint32_t nrows = 2 * s.k - 1;
    hipError_t e = launch_rows(s.M, K, src, tr, 0, true, st);
    if (e == hipSuccess) e = launch_cols(s.R, K, tr, s.M, s.k, st);
    if (e == hipSuccess) e = launch_rows(s.M, K, src, tr, 2 * nrows, false, st);
    if (e != hipSuccess) return e;
    // L, H and the tile statuses, then L + H with each tile's carry-in
    // derived from the statuses below it
    const uint64_t nwords = 2 * n32, ntiles = (nwords + kLargeTileWords - 1) / kLargeTileWords;
    auto *status = scratch + s.st;
    const LargeCoef coef{tr, 1u << s.M, 2 * bw, nrows, K.p[0], K.p[1], K.crt, K.crt_sh};
    const uint32_t grid = uint32_t(std::min<uint64_t>(ntiles, 65536));
    hipLaunchKernelGGL(large_ntt_fold_kernel, dim3(grid), dim3(256), 0, st, coef, nwords, Lw, Hw, status);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(large_ntt_add_kernel, dim3(grid), dim3(256), 0, st, Lw, Hw, status, out, uint32_t(nwords));
    return hipGetLastError();
}

}  // namespace bi
