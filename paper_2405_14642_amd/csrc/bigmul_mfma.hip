// Schoolbook multiplication on int8 matrix cores (the convolution of eq. (1)
// in Section 3.1, re-expressed for v_mfma_i32_32x32x32_i8).
//
// Digits.  An operand of n32 32-bit limbs, padded to n32p (a multiple of 8),
// is D = 4 n32p bytes.  Adding R = 0x8080...80 (one D-byte addition with a
// carry scan) and flipping the top bit of every byte gives balanced digits
// d_i = byte_i(A + R) - 128 in [-128, 127] with A = sum d_i 256^i + t 256^D,
// t in {0, 1} the carry out.  The D x D digit convolution has
// |c_k| <= D 2^14, and the cross terms t_A b_j + t_B a_j at k = D + j add at
// most 2^8, so int32 accumulation cannot overflow for D <= 2^15.  The term
// t_A t_B 256^(2D) lies above the product's 2D bytes and is dropped.
//
// Block Toeplitz form.  With output blocks of 32 coefficients,
//   C[32 K + r] = sum_{u=0..nb} sum_{s<32} a[32 u + r - s] b[32 (K - u) + s]
// (nb = D / 32; digits outside [0, D) are zero), so for a fixed u one
// 32 x 32 x 32 MFMA with A operand T_u[r][s] = a[32 u + r - s] and B operand
// "digit blocks K - u of b, K = 32 st .. 32 st + 31" adds the u-th term to
// the 32 output blocks of supertile st.  The k index of both operands runs
// through s in reverse inside each 16-byte half, so lane (r, g) reads
// a[32 u + r - 16 g - 15 ..] as 16 ascending bytes: from one of 8 byte-shifted
// copies of a, at an 8-byte aligned address (one ds_read2_b64).  b is stored
// with every 16-digit group byte-reversed, the two halves of each 32-digit
// block in separate planes, so the B reads of a wave are contiguous.
//
// Work split.  Supertile st needs the u in [32 st - nb + 1, 32 st + 31]
// clipped to [0, nb]; supertiles st and st + h (h = half their number) need
// about nb + 32 steps together, so each wave owns such a pair, keeps its
// accumulators in registers and needs no atomics.
//
// Normalisation.  A lane holds, for each of its output words w, the four
// coefficients of bytes 4w .. 4w+3.  V_w = sum_e c_e 2^(8e) + 2^63 - 2^31 [w > 0]
// is in [0, 2^64); its low word goes to L[w], its high word to H[w + 1].  The
// biases cancel between neighbouring words except 2^63 at the top word, which
// lies above the product.  L + H is added with the workgroup ballot-adder, as
// for the other products (Section 3.1 combines its low and high parts the
// same way).
#include "bi_common.hpp"
#include "bi_internal.hpp"
#include "bi_wgadd.hpp"

namespace bi {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr uint32_t kPA = 40;     // zero bytes before the digits of a in copy 0
constexpr uint32_t kBPad = 32;   // zero B entries before block 0
constexpr uint32_t kBTail = 31;  // zero B entries after the last block
constexpr uint32_t kR8 = 0x80808080u;

struct MfmaLayout {  // byte offsets into the dynamic LDS block
    uint32_t D, nb, CSA, NBE;
    uint32_t bpl, sum, total;
};

__host__ __device__ inline MfmaLayout mfma_layout(uint32_t n32p) {
    MfmaLayout l;
    l.D = 4 * n32p;
    l.nb = l.D / 32;
    // Copy stride: the MFMA loop reads copy bytes below kPA + D + 64 and the
    // last 16-byte chunk of a copy is never built, so the stride is at least
    // kPA + D + 80; = 32 mod 128 spreads the 8 copies over the LDS banks.
    l.CSA = ((kPA + l.D + 48 + 127) / 128) * 128 + 32;
    l.NBE = kBPad + l.nb + kBTail;
    l.bpl = 8 * l.CSA;
    l.sum = l.bpl + 2 * 16 * l.NBE;
    l.total = l.sum + 3 * 16;
    return l;
}

// Low words L[w] and high words H[w] (H[0] = 0), both in LDS.
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

}  // namespace

template <int NW, class Src>
__global__ __launch_bounds__(64 * NW) void bigmul_mfma_kernel(Src src) {
    extern __shared__ __align__(16) uint8_t lds[];
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = wave_in_block();
    constexpr uint32_t T = 64 * NW;
    const uint64_t count = src.count();

    for (uint64_t pair = blockIdx.x; pair < count; pair += gridDim.x) {
        const InstRef in = src.get(pair);
        const uint32_t n32 = in.n, n32p = (n32 + 7) & ~7u;
        const MfmaLayout lo = mfma_layout(n32p);
        const uint32_t D = lo.D, nb = lo.nb, CSA = lo.CSA, NBE = lo.NBE;
        uint8_t *bpl = lds + lo.bpl;
        uint32_t *summary = reinterpret_cast<uint32_t *>(lds + lo.sum);

        // 1. balanced digits: a in natural order into copy 0, b group-reversed
        //    into the two B planes; zero the pads around both.
        const uint32_t *a = in.a, *b = in.b;
        auto src_a = [&](uint32_t c, uint32_t (&x)[4], uint32_t (&y)[4]) {
            load4(a, n32, c, x);
            y[0] = y[1] = y[2] = y[3] = kR8;
        };
        auto sink_a = [&](uint32_t c, const uint32_t (&s)[4]) {
            uint64_t *p = reinterpret_cast<uint64_t *>(lds + kPA + 16 * c);
            p[0] = uint64_t(s[0] ^ kR8) | (uint64_t(s[1] ^ kR8) << 32);
            p[1] = uint64_t(s[2] ^ kR8) | (uint64_t(s[3] ^ kR8) << 32);
        };
        const uint32_t tA = wg_add_rows_sink<NW>(src_a, sink_a, n32p, summary);
        auto src_b = [&](uint32_t c, uint32_t (&x)[4], uint32_t (&y)[4]) {
            load4(b, n32, c, x);
            y[0] = y[1] = y[2] = y[3] = kR8;
        };
        auto sink_b = [&](uint32_t c, const uint32_t (&s)[4]) {
            uint4 v;
            v.x = __builtin_bswap32(s[3] ^ kR8);
            v.y = __builtin_bswap32(s[2] ^ kR8);
            v.z = __builtin_bswap32(s[1] ^ kR8);
            v.w = __builtin_bswap32(s[0] ^ kR8);
            *reinterpret_cast<uint4 *>(bpl + (c & 1u) * 16 * NBE + 16 * (kBPad + (c >> 1))) = v;
        };
        const uint32_t tB = wg_add_rows_sink<NW>(src_b, sink_b, n32p, summary + 4);
        {
            uint64_t *a0 = reinterpret_cast<uint64_t *>(lds);
            const uint32_t z0 = kPA / 8, z1 = (kPA + D) / 8, z2 = CSA / 8;
            for (uint32_t i = tid; i < z0 + (z2 - z1); i += T) a0[i < z0 ? i : z1 + (i - z0)] = 0;
            const uint32_t nz = kBPad + kBTail;
            for (uint32_t i = tid; i < 2 * nz; i += T) {
                const uint32_t pl = i / nz, e = i - pl * nz;
                const uint32_t ent = e < kBPad ? e : nb + e;
                *reinterpret_cast<uint4 *>(bpl + pl * 16 * NBE + 16 * ent) = make_uint4(0, 0, 0, 0);
            }
        }
        __syncthreads();

        // 2. copies 1..7: copy c byte y = copy 0 byte y + c
        {
            const uint32_t nq = CSA / 16 - 1;
            for (uint32_t c = 1; c < 8; ++c) {
                for (uint32_t q = tid; q < nq; q += T) {
                    const uint4 x0 = *reinterpret_cast<const uint4 *>(lds + 16 * q);
                    const uint4 x1 = *reinterpret_cast<const uint4 *>(lds + 16 * q + 16);
                    const uint32_t w[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
                    const uint32_t o = c >> 2, sh = c & 3u;
                    uint4 v;
                    v.x = __builtin_amdgcn_alignbyte(w[o + 1], w[o + 0], sh);
                    v.y = __builtin_amdgcn_alignbyte(w[o + 2], w[o + 1], sh);
                    v.z = __builtin_amdgcn_alignbyte(w[o + 3], w[o + 2], sh);
                    v.w = __builtin_amdgcn_alignbyte(w[o + 4], w[o + 3], sh);
                    *reinterpret_cast<uint4 *>(lds + c * CSA + 16 * q) = v;
                }
            }
        }
        __syncthreads();

        // 3. MFMA: this wave's supertiles wave and wave + h
        const uint32_t nst = (n32p + 127) / 128, h = (nst + 1) / 2;
        const uint32_t r = lane & 31u, g = lane >> 5;
        uint32_t Lo[2][4], Hi[2][4];
        const uint32_t xb = r + kPA - 16 * g - 15, cpy = xb & 7u;
        const uint8_t *abase = lds + cpy * CSA + (xb - cpy);
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const uint32_t st = wave + uint32_t(t) * h;
            if (wave >= h || st >= nst) continue;
            const int32_t ulo = max(0, int32_t(32 * st) - int32_t(nb) + 1);
            const int32_t uhi = min(int32_t(nb), int32_t(32 * st + 31));
            const uint8_t *bbase = bpl + g * 16 * NBE + 16 * (32 * st + r + kBPad);
            auto ldA = [&](int32_t u) -> v4i {
                const uint64_t *p = reinterpret_cast<const uint64_t *>(abase + 32 * u);
                const uint64_t x0 = p[0], x1 = p[1];
                return v4i{int(uint32_t(x0)), int(uint32_t(x0 >> 32)), int(uint32_t(x1)), int(uint32_t(x1 >> 32))};
            };
            auto ldB = [&](int32_t u) -> v4i { return *reinterpret_cast<const v4i *>(bbase - 16 * u); };
            v16i acc0 = {}, acc1 = {};
            const int32_t npair = (uhi - ulo + 2) >> 1;
            int32_t u = ulo;
            v4i a0 = ldA(u), b0 = ldB(u), a1 = ldA(u + 1), b1 = ldB(u + 1);
            for (int32_t i = 0; i < npair; ++i) {
                const int32_t un = (i + 1 < npair) ? u + 2 : u;
                const v4i na0 = ldA(un), nb0 = ldB(un), na1 = ldA(un + 1), nb1 = ldB(un + 1);
                acc0 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0, b0, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1, b1, acc1, 0, 0, 0);
                a0 = na0; b0 = nb0; a1 = na1; b1 = nb1;
                u = un;
            }
            // acc[4j + i] at lane (r, g) is coefficient 32 K + 8 j + 4 g + i,
            // K = 32 st + r: the four bytes of word w = 8 K + 2 j + g.
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t w = 256 * st + 8 * r + 2 * uint32_t(j) + g;
                int32_t c[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) c[e] = acc0[4 * j + e] + acc1[4 * j + e];
                if (w >= n32p && w < 2 * n32p && (tA | tB)) {
                    const uint32_t m = w - n32p, cc = m >> 2;
                    const uint32_t aw = *reinterpret_cast<const uint32_t *>(lds + kPA + 4 * m);
                    const uint32_t bw = *reinterpret_cast<const uint32_t *>(
                        bpl + (cc & 1u) * 16 * NBE + 16 * (kBPad + (cc >> 1)) + 4 * (3 - (m & 3u)));
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        c[e] += int32_t(tA) * sbyte(bw, 3 - e) + int32_t(tB) * sbyte(aw, e);
                }
                uint64_t V = uint64_t(int64_t(c[0])) + (uint64_t(int64_t(c[1])) << 8) +
                             (uint64_t(int64_t(c[2])) << 16) + (uint64_t(int64_t(c[3])) << 24);
                V += (1ull << 63) - (w > 0 ? (1ull << 31) : 0ull);
                Lo[t][j] = uint32_t(V);
                Hi[t][j] = uint32_t(V >> 32);
            }
        }
        __syncthreads();  // every wave is done with the copies of a

        // 4. L and H (aliasing the copies), then product = L + H
        const uint32_t W = 2 * n32p;
        uint32_t *L = reinterpret_cast<uint32_t *>(lds);
        uint32_t *H = L + W;
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const uint32_t st = wave + uint32_t(t) * h;
            if (wave >= h || st >= nst) continue;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t w = 256 * st + 8 * r + 2 * uint32_t(j) + g;
                if (w < W) L[w] = Lo[t][j];
                if (w + 1 < W) H[w + 1] = Hi[t][j];
            }
        }
        if (tid == 0) H[0] = 0;
        __syncthreads();
        wg_add_rows<NW>(LHSrc{L, H, 2 * n32}, in.c, 2 * n32, summary + 8);
        __syncthreads();
    }
}

uint32_t mfma_max_limbs() { return 1024; }

// Waves per workgroup: one per pair of supertiles (1024 output digits each).
static uint32_t mfma_waves(uint32_t nmax) {
    const uint32_t n32p = (nmax + 7) & ~7u;
    const uint32_t nst = (n32p + 127) / 128, h = (nst + 1) / 2;
    return h <= 1 ? 1 : h <= 2 ? 2 : 4;
}

template <int NW, class Src>
static hipError_t launch_nw(const Src &src, uint32_t nmax, uint64_t count, hipStream_t st) {
    const MfmaLayout lo = mfma_layout((nmax + 7) & ~7u);
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&bigmul_mfma_kernel<NW, Src>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr = true;
    }
    const uint32_t grid = uint32_t(count < 65536 ? count : 65536);
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL((bigmul_mfma_kernel<NW, Src>), dim3(grid), dim3(64 * NW), lo.total, st, src);
    return hipGetLastError();
}

template <class Src>
static hipError_t launch_mfma(const Src &src, uint32_t nmax, uint64_t count, hipStream_t st) {
    if (nmax > mfma_max_limbs()) return hipErrorInvalidValue;
    switch (mfma_waves(nmax)) {
        case 1: return launch_nw<1>(src, nmax, count, st);
        case 2: return launch_nw<2>(src, nmax, count, st);
        default: return launch_nw<4>(src, nmax, count, st);
    }
}

hipError_t launch_bigmul_mfma(const uint32_t *a, const uint32_t *b, uint32_t *c, uint32_t n32, uint64_t batch,
                              hipStream_t st) {
    if (batch == 0) return hipSuccess;
    return launch_mfma(UniformInst{a, b, c, n32, batch}, n32, batch, st);
}

hipError_t launch_bigmul_mfma_list(const ListInst &src, uint32_t nmax, uint64_t count_max, hipStream_t st) {
    return launch_mfma(src, nmax, count_max, st);
}

}  // namespace bi
