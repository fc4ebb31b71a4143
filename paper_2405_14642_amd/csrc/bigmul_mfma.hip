// Schoolbook multiplication on int8 matrix cores (the convolution of eq. (1)
// in Section 3.1, re-expressed for v_mfma_i32_32x32x32_i8).
//
// Digits.  An operand of n32 32-bit limbs is D = 4 n32 bytes.  Adding
// R = 0x8080...80 (one D-byte addition with a carry scan) and flipping the top
// bit of every byte gives balanced digits d_i = byte_i(A + R) - 128 in
// [-128, 127] with A = sum d_i 256^i + t 256^D, t in {0, 1} the carry out.
// The D x D digit convolution has |c_k| <= D 2^14 and the two cross terms
// t_A b_j, t_B a_j at k = D + j at most 2^8 more, so every coefficient stays
// below 2^29 for D <= 2^15 and the int32 accumulators cannot overflow.
//
// Block Toeplitz form.  With output blocks of 32 coefficients,
//   C[32 K + r] = sum_u sum_{s<32} T_u[r][s] b[32 (K - u) + s],
//   T_u[r][s]   = a[32 u + r - s]  (zero outside [0, D)),
// so for a fixed u a 32 x 32 x 32 MFMA with A operand T_u and B operand
// "digit blocks K0-u .. K0-u+31 of b" adds the u-th term to 32 consecutive
// output blocks (a supertile).  Row r of T_u is a reversed window of a: the
// workgroup keeps 16 copies of the reversed digit string shifted by 0..15
// bytes, so every lane reads its 16-byte window with one aligned LDS read.
// Work items are (supertile, run of 16 u), spread over the waves; each adds
// its 32 x 32 tile into the LDS coefficient array with LDS atomics.
//
// Normalisation.  Groups of 16 signed coefficients are folded into 4 low words
// and one high word; adding 2^31 to every group's high word (and taking 2^31
// from the next group's low word) makes all words non-negative while changing
// the total only above the product's top word.  The low and high arrays are
// then added with the workgroup ballot-adder, as for the other products.
#include "bi_common.hpp"
#include "bi_internal.hpp"
#include "bi_wgadd.hpp"

namespace bi {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr uint32_t kPadA = 35;  // reversed string offset X = D + 35 (X = 3 mod 4)
constexpr uint32_t kUch = 16;   // u-steps per work item

struct MfmaLayout {  // byte offsets into the dynamic LDS block
    uint32_t D, nb, CS, G;
    uint32_t acopy, bdig, coef, small, total;
};

__host__ __device__ inline MfmaLayout mfma_layout(uint32_t n32p) {
    MfmaLayout l;
    l.D = 4 * n32p;
    l.nb = l.D / 32;
    // copy stride: >= D + 80 bytes, = 16 mod 256 so the 16 copies' windows at
    // the same offset fall into distinct banks
    l.CS = ((l.D + 80 + 255) / 256) * 256 + 16;
    l.G = (2 * l.D + 1 + 15) / 16;  // normalisation groups of 16 coefficients
    l.acopy = 0;
    l.bdig = 16 * l.CS;
    l.coef = l.bdig + l.D;
    l.small = l.coef + 4 * (2 * l.D + 16);
    l.total = l.small + 4 * 32;
    return l;
}

// One word per group at word position 4 (g+1) (the high word of group g).
struct LHSrc4w1 {
    const uint32_t *L;
    const uint32_t *H;
    uint32_t nwords;
    __device__ __forceinline__ void operator()(uint32_t c, uint32_t (&x)[4], uint32_t (&y)[4]) const {
        const uint4 l = *reinterpret_cast<const uint4 *>(L + 4 * c);
        x[0] = l.x; x[1] = l.y; x[2] = l.z; x[3] = l.w;
        if (c >= 1) y[0] = H[c - 1];
        const uint32_t base = 4 * c;
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if (base + t >= nwords) { x[t] = 0; y[t] = 0; }
    }
};

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
        const uint32_t *a = in.a;
        const uint32_t *b = in.b;
        const MfmaLayout lo = mfma_layout(n32p);
        uint8_t *acopy = lds + lo.acopy;
        uint8_t *bdig = lds + lo.bdig;
        int32_t *coef = reinterpret_cast<int32_t *>(lds + lo.coef);
        uint32_t *adig = reinterpret_cast<uint32_t *>(lds + lo.coef);  // temporary, aliases coef
        uint32_t *summary = reinterpret_cast<uint32_t *>(lds + lo.small);
        uint32_t *Lw = reinterpret_cast<uint32_t *>(lds + lo.acopy);  // normalisation, aliases the copies
        uint32_t *Hw = Lw + 4 * lo.G;
        const uint32_t D = lo.D, nb = lo.nb, CS = lo.CS, X = D + kPadA;

        // 1. balanced digits of a (words of (a + R) ^ R) and its top digit
        auto src_a = [&](uint32_t c, uint32_t (&x)[4], uint32_t (&y)[4]) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const uint32_t w = 4 * c + t;
                x[t] = w < n32 ? a[w] : 0u;
                y[t] = 0x80808080u;
            }
        };
        auto sink_a = [&](uint32_t c, const uint32_t (&s)[4]) {
#pragma unroll
            for (int t = 0; t < 4; ++t) adig[4 * c + t] = s[t] ^ 0x80808080u;
        };
        const uint32_t tA = wg_add_rows_sink<NW>(src_a, sink_a, n32p, summary);
        __syncthreads();

        // 2. 16 copies of the reversed digit string R[x] = a[X - x]; copy c holds
        //    R[y + c] at byte y.  Word q of copy c is a[i0 .. i0+3] reversed,
        //    i0 = X - 4q - c - 3.
        for (uint32_t idx = tid; idx < 16 * (CS / 4); idx += T) {
            const uint32_t c = idx / (CS / 4), q = idx - c * (CS / 4);
            const int32_t i0 = int32_t(X) - int32_t(4 * q + c + 3);
            const int32_t w0 = i0 >> 2;  // floor
            const uint32_t sh = uint32_t(i0) & 3u;
            const uint32_t lo_w = (w0 >= 0 && w0 < int32_t(n32p)) ? adig[w0] : 0u;
            const uint32_t hi_w = (w0 + 1 >= 0 && w0 + 1 < int32_t(n32p)) ? adig[w0 + 1] : 0u;
            const uint32_t v = uint32_t(((uint64_t(hi_w) << 32) | lo_w) >> (8 * sh));
            *reinterpret_cast<uint32_t *>(acopy + c * CS + 4 * q) = __builtin_bswap32(v);
        }

        // 3. balanced digits of b, in natural order
        auto src_b = [&](uint32_t c, uint32_t (&x)[4], uint32_t (&y)[4]) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const uint32_t w = 4 * c + t;
                x[t] = w < n32 ? b[w] : 0u;
                y[t] = 0x80808080u;
            }
        };
        uint32_t *bw = reinterpret_cast<uint32_t *>(bdig);
        auto sink_b = [&](uint32_t c, const uint32_t (&s)[4]) {
#pragma unroll
            for (int t = 0; t < 4; ++t) bw[4 * c + t] = s[t] ^ 0x80808080u;
        };
        const uint32_t tB = wg_add_rows_sink<NW>(src_b, sink_b, n32p, summary);
        __syncthreads();  // copies built, adig dead
        for (uint32_t k = tid; k < 2 * D + 16; k += T) coef[k] = 0;
        __syncthreads();

        // 4. MFMA work items (supertile st, chunk ch of its u-range)
        const uint32_t nst = (2 * nb + 31) / 32;
        {
            const uint32_t r = lane & 31u, g = lane >> 5;
            uint32_t item = wave, base = 0;
            for (uint32_t st = 0; st < nst; ++st) {
                const int32_t ulo = max(0, int32_t(32 * st) - int32_t(nb) + 1);
                const int32_t uhi = min(int32_t(nb), int32_t(32 * st + 31));
                const uint32_t cnt = uint32_t(uhi - ulo + int32_t(kUch)) / kUch;
                for (; item < base + cnt; item += NW) {
                    const int32_t u0 = ulo + int32_t((item - base) * kUch);
                    const int32_t u1 = min(uhi, u0 + int32_t(kUch) - 1);
                    v16i acc0 = {}, acc1 = {};
                    for (int32_t u = u0; u <= u1; ++u) {
                        const uint32_t x0 = X - 32 * uint32_t(u) - r + 16 * g;
                        const uint32_t cc = x0 & 15u;
                        const v4i av = *reinterpret_cast<const v4i *>(acopy + cc * CS + (x0 - cc));
                        const int32_t blk = int32_t(32 * st + r) - u;  // lane's column is r (= lane mod 32)
                        v4i bv = {0, 0, 0, 0};
                        if (blk >= 0 && blk < int32_t(nb)) bv = *reinterpret_cast<const v4i *>(bdig + 32 * blk + 16 * g);
                        if ((u - u0) & 1)
                            acc1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(av, bv, acc1, 0, 0, 0);
                        else
                            acc0 = __builtin_amdgcn_mfma_i32_32x32x32_i8(av, bv, acc0, 0, 0, 0);
                    }
                    // acc[i] at lane l: row 8 (i/4) + 4 (l/32) + i%4, column l%32
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        const uint32_t row = 8 * (i / 4) + 4 * g + (i % 4);
                        const uint32_t k = 32 * (32 * st + r) + row;
                        if (k < 2 * D) atomicAdd(&coef[k], acc0[i] + acc1[i]);
                    }
                }
                base += cnt;
            }
        }
        __syncthreads();

        // 5. top digits: t_A b 256^D + t_B a 256^D + t_A t_B 256^(2D)
        for (uint32_t j = tid; j < D; j += T) {
            const int32_t da = int32_t(int8_t(acopy[X - j]));  // copy 0: R[X - j] = a[j]
            const int32_t db = int32_t(int8_t(bdig[j]));
            coef[D + j] += int32_t(tA) * db + int32_t(tB) * da;
        }
        if (tid == 0) coef[2 * D] += int32_t(tA & tB);
        __syncthreads();

        // 6. groups of 16 coefficients -> 4 low words + 1 biased high word
        for (uint32_t gi = tid; gi < lo.G; gi += T) {
            int64_t col[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                col[j] = 0;
#pragma unroll
                for (int e = 0; e < 4; ++e) col[j] += int64_t(coef[16 * gi + 4 * j + e]) * (int64_t(1) << (8 * e));
            }
            if (gi > 0) col[0] -= int64_t(1) << 31;
            int64_t carry = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t xv = col[j] + carry;
                Lw[4 * gi + j] = uint32_t(uint64_t(xv));
                carry = xv >> 32;  // arithmetic: floor division
            }
            Hw[gi] = uint32_t(carry + (int64_t(1) << 31));
        }
        __syncthreads();

        // 7. product = L + H (mod 2^(64 n32))
        wg_add_rows<NW>(LHSrc4w1{Lw, Hw, 2 * n32}, in.c, 2 * n32, summary);
        __syncthreads();
    }
}

uint32_t mfma_max_limbs() { return 1024; }

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
    if (nmax <= 256) return launch_nw<4>(src, nmax, count, st);
    return launch_nw<8>(src, nmax, count, st);
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
