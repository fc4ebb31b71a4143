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
// a[32 u + r - 16 g - 15 ..] as 16 ascending bytes.  LDS holds every 8-byte
// window of a's digits: entry x (8 bytes at 8 x) = digits x - kPA .. x - kPA + 7,
// so the lanes of a wave read consecutive entries x and x + 8 (two
// conflict-free 8-byte reads) whatever the byte offset.  b is stored with
// every 16-digit group byte-reversed, the two halves of each 32-digit block in
// separate planes, so the B reads of a wave are contiguous too.
//
// Work split.  Supertile st needs the u in [32 st - nb + 1, 32 st + 31]
// clipped to [0, nb].  Each wave owns two adjacent supertiles, whose ranges
// coincide but for 32 steps at each end, keeps their accumulators in
// registers (no atomics), and reads each A operand once for both: three
// 1 KiB LDS reads per two MFMAs, the traffic that bounds the loop.
//
// 1024-limb products (nb = 128, eight supertiles) and 512-limb products
// (nb = 64, four supertiles) take a k-major order instead.  Since B(st + i, u) = B(st, u - 32 i), a wave that owns four
// consecutive supertiles sb + i and walks u = k + 32 m with the residue k
// outer needs one A operand per m and one B operand beta_j = B(sb, k + 32 j)
// per j: supertile sb + i at m takes A(k + 32 m) and beta_(m - i), so each
// read serves up to four MFMAs (0.8 KiB per MFMA).  At nb = 128 the in-band
// (i, m) of every residue form a fixed triangle: m <= i for supertiles 0-3
// (k = 0 .. 31), m >= i for supertiles 4-7 (k = 1 .. 32); at nb = 64 the
// four supertiles form one group whose (i, m) are fixed for k = 1 .. 31.
// The two waves of a group take alternate residues and each finalises two of the four
// supertiles, adding the other wave's 64-bit partial word sums, passed
// through LDS, to its own.
//
// Normalisation.  A lane holds, for each of its output words w, the four
// coefficients of bytes 4w .. 4w+3.  V_w = sum_e c_e 2^(8e) + 2^63 - 2^31 [w > 0]
// is in [0, 2^64); its low word goes to L[w], its high word to H[w + 1].  The
// biases cancel between neighbouring words except 2^63 at the top word, which
// lies above the product.  L + H is added with the workgroup ballot-adder, as
// for the other products (Section 3.1 combines its low and high parts the
// same way).
#include <algorithm>
#include <atomic>

#include "bi_common.hpp"
#include "bi_internal.hpp"
#include "bi_mfma.hpp"
#include "bi_wgadd.hpp"

namespace bi {

namespace {

using namespace mfma;

constexpr uint32_t kPA = 32;     // zero bytes before the digits of a
constexpr uint32_t kBPad = 32;   // zero B entries before block 0
constexpr uint32_t kBTail = 31;  // zero B entries after the last block

struct MfmaLayout {  // byte offsets into the dynamic LDS block
    uint32_t D, nb, NE, NBE, bpad;  // bpad: zero B entries before block 0
    uint32_t a0, A0S, bpl, sum, total;
};

// one: products of a single supertile (n32p <= 128, one wave), whose B reads
// cover blocks -16 .. 31 and whose A reads stay below window D + 57: a
// layout of 6.8 KB at 128 limbs (six workgroups per SIMD) instead of 8.1.
__host__ __device__ inline MfmaLayout mfma_layout(uint32_t n32p, bool one = false) {
    MfmaLayout l;
    l.D = 4 * n32p;
    l.nb = l.D / 32;
    // 8-byte windows: the MFMA loop reads entries below D + 89 (D + 57 with
    // one supertile)
    l.NE = ((one ? l.D + 57 : l.D + 89) + 31) & ~31u;
    // digits of a with kPA zero bytes before and zeros up to NE + 16
    l.a0 = 8 * l.NE;
    l.A0S = (l.NE + 16 + 15) & ~15u;
    l.bpad = one ? 16u : kBPad;
    l.NBE = one ? 48u : kBPad + l.nb + kBTail;
    l.bpl = l.a0 + l.A0S;
    l.sum = l.bpl + 2 * 16 * l.NBE;
    l.total = l.sum + 3 * 16;
    return l;
}

// Operand words of one 16-byte chunk per lane: chunk c = 64 w + lane of wave
// w (zero beyond n words).
struct Chunks {
    uint32_t a[4];
    uint32_t b[4];
};

__device__ __forceinline__ void fetch_chunks(const InstRef &in, uint32_t c, Chunks &x) {
    load4(in.a, in.n, c, x.a);
    load4(in.b, in.n, c, x.b);
}

// Balanced digits of both operands in one carry scan per operand (nchunks <=
// 64 NW, one chunk per lane).  On return x.a / x.b hold the digit words of
// (A + R) ^ R and t[0], t[1] the carries t_A, t_B.
template <int NW>
__device__ __forceinline__ void recode_chunks(Chunks &x, uint32_t nchunks, uint32_t *summary, uint32_t (&t)[2]) {
    const uint32_t lane = lane_id(), w = wave_in_block();
    const uint32_t c = 64 * w + lane;
    const uint32_t valid = nchunks > 64 * w ? min(nchunks - 64 * w, 64u) : 0u;
    const uint64_t vmask = valid >= 64 ? ~0ull : ((1ull << valid) - 1);
    const uint32_t R[4] = {kR8, kR8, kR8, kR8};
    uint32_t sa[4], sb[4];
    const uint32_t ga = add_words<4>(x.a, R, sa);
    const uint32_t gb = add_words<4>(x.b, R, sb);
    const uint64_t Ga = ballot(ga != 0), Pa = ballot(c < nchunks && all_ones<4>(sa));
    const uint64_t Gb = ballot(gb != 0), Pb = ballot(c < nchunks && all_ones<4>(sb));
    // carries out of this wave's chunks; one wave: the operands' carries
    const WaveCarry ca0 = wave_carry(Ga, Pa, 0), cb0 = wave_carry(Gb, Pb, 0);
    const uint32_t oa = valid >= 64 ? ca0.out : uint32_t(ca0.into >> valid) & 1u;
    const uint32_t ob = valid >= 64 ? cb0.out : uint32_t(cb0.into >> valid) & 1u;
    uint32_t cina = 0, cinb = 0, ta = oa, tb = ob;
    if constexpr (NW > 1) {
        if (lane == 0) {
            summary[w] = oa | ((Pa == vmask ? 1u : 0u) << 1);
            summary[4 + w] = ob | ((Pb == vmask ? 1u : 0u) << 1);
        }
        __syncthreads();
        ta = tb = 0;
#pragma unroll
        for (uint32_t v = 0; v < uint32_t(NW); ++v) {
            const uint32_t sva = summary[v], svb = summary[4 + v];
            if (v < w) {
                cina = (sva & 1u) | ((sva >> 1) & cina);
                cinb = (svb & 1u) | ((svb >> 1) & cinb);
            }
            ta = (sva & 1u) | ((sva >> 1) & ta);
            tb = (svb & 1u) | ((svb >> 1) & tb);
        }
    }
    t[0] = ta;
    t[1] = tb;
    const WaveCarry ca = wave_carry(Ga, Pa, cina), cb = wave_carry(Gb, Pb, cinb);
    add_carry_words<4>(sa, uint32_t(ca.into >> lane) & 1u);
    add_carry_words<4>(sb, uint32_t(cb.into >> lane) & 1u);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        x.a[i] = sa[i] ^ kR8;
        x.b[i] = sb[i] ^ kR8;
    }
}

// k-major MFMA steps of a 1024-limb product for one group of four
// supertiles sb .. sb + 3 (HIGH: sb = 4), residues k = k0, k0 + 2, ...
// bbs: this lane's B entry of supertile sb at step 0.  Supertile sb + i
// accumulates into acc[i ^ X]: with X = 2 the second wave of the group also
// holds the two supertiles it finalises in acc[0..1].  Every read lies in
// band, hence inside the padded arrays.
template <bool HIGH, int X>
__device__ __forceinline__ void mfma_kmajor_1024(const uint8_t *lds, uint32_t oA, const uint8_t *bbs, int32_t k0,
                                                 v16i (&acc)[4]) {
    constexpr int32_t J0 = HIGH ? 0 : -3;  // beta_j for j = J0 .. J0 + 3
    for (int32_t k = k0; k < (HIGH ? 33 : 32); k += 2) {
        v4i A[4], Bt[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) A[m] = load_a(lds, oA, k + 32 * m);
#pragma unroll
        for (int j = 0; j < 4; ++j) Bt[j] = *reinterpret_cast<const v4i *>(bbs - 16 * (k + 32 * (j + J0)));
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (HIGH ? m >= i : m <= i)
                    acc[i ^ X] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[m], Bt[m - i - J0], acc[i ^ X], 0, 0, 0);
    }
}

// k-major MFMA steps of a 512-limb product (nb = 64: supertiles 0 .. 3, one
// group of two waves), residues k = k0, k0 + 2, .. 31.  At k = 1 .. 31
// supertile i takes u = k + 32 m for m in [max(0, i - 2), min(i, 1)], whose
// B is beta_(m - i): two A and three B reads feed six MFMAs.  Residue 0 takes
// u = 0, 32, 64 instead (m = 2 lies in band for supertiles 2 and 3 only
// there, and u = 0 / u = 32 leave the bands of supertiles 2 / 3).
template <int X>
__device__ __forceinline__ void mfma_kmajor_512(const uint8_t *lds, uint32_t oA, const uint8_t *bbs, int32_t k0,
                                                v16i (&acc)[4]) {
    auto beta = [bbs](int32_t k, int32_t j) { return *reinterpret_cast<const v4i *>(bbs - 16 * (k + 32 * j)); };
    // operands of residue k: A(k), A(k + 32), beta_0, beta_-1, beta_-2
    auto operands = [&](int32_t k, v4i (&o)[5]) {
        o[0] = load_a(lds, oA, k);
        o[1] = load_a(lds, oA, k + 32);
        o[2] = beta(k, 0);
        o[3] = beta(k, -1);
        o[4] = beta(k, -2);
    };
    int32_t k = k0;
    if (k0 == 0) {
        const v4i A0 = load_a(lds, oA, 0), A1 = load_a(lds, oA, 32), A2 = load_a(lds, oA, 64);
        const v4i b0 = beta(0, 0), b1 = beta(0, -1);
        acc[0 ^ X] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A0, b0, acc[0 ^ X], 0, 0, 0);
        acc[1 ^ X] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A0, b1, acc[1 ^ X], 0, 0, 0);
        acc[1 ^ X] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A1, b0, acc[1 ^ X], 0, 0, 0);
        acc[2 ^ X] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A1, b1, acc[2 ^ X], 0, 0, 0);
        acc[2 ^ X] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A2, b0, acc[2 ^ X], 0, 0, 0);
        acc[3 ^ X] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A2, b1, acc[3 ^ X], 0, 0, 0);
        k = 2;
    }
#pragma unroll 1
    for (; k < 32; k += 2) {
        v4i o[5];
        operands(k, o);
        acc[0 ^ X] = __builtin_amdgcn_mfma_i32_32x32x32_i8(o[0], o[2], acc[0 ^ X], 0, 0, 0);
        acc[1 ^ X] = __builtin_amdgcn_mfma_i32_32x32x32_i8(o[0], o[3], acc[1 ^ X], 0, 0, 0);
        acc[1 ^ X] = __builtin_amdgcn_mfma_i32_32x32x32_i8(o[1], o[2], acc[1 ^ X], 0, 0, 0);
        acc[2 ^ X] = __builtin_amdgcn_mfma_i32_32x32x32_i8(o[0], o[4], acc[2 ^ X], 0, 0, 0);
        acc[2 ^ X] = __builtin_amdgcn_mfma_i32_32x32x32_i8(o[1], o[3], acc[2 ^ X], 0, 0, 0);
        acc[3 ^ X] = __builtin_amdgcn_mfma_i32_32x32x32_i8(o[1], o[4], acc[3 ^ X], 0, 0, 0);
    }
}

// Lane-order mask (lane r + 32 g) to chunk order (chunk 2 r + g).
__device__ __forceinline__ uint64_t lanes_to_chunks(uint64_t m) {
    auto spread = [](uint32_t x) {
        uint64_t v = x;
        v = (v | (v << 16)) & 0x0000FFFF0000FFFFull;
        v = (v | (v << 8)) & 0x00FF00FF00FF00FFull;
        v = (v | (v << 4)) & 0x0F0F0F0F0F0F0F0Full;
        v = (v | (v << 2)) & 0x3333333333333333ull;
        return (v | (v << 1)) & 0x5555555555555555ull;
    };
    return spread(uint32_t(m)) | (spread(uint32_t(m >> 32)) << 1);
}

// Sum_e c_e 2^(8e) of output word j of a lane's accumulator block.
__device__ __forceinline__ int64_t word_sum(const v16i &a, int j) {
    return int64_t(a[4 * j]) + (int64_t(a[4 * j + 1]) << 8) + (int64_t(a[4 * j + 2]) << 16) +
           (int64_t(a[4 * j + 3]) << 24);
}

// Byte offset of the partial-sum exchange between the two waves of a group
// (NW * 4 KiB: per wave 2 supertiles x 4 words x 64 lanes x 8 bytes): the
// windows of a, dead by then, when they are large enough, else past the
// layout.
__host__ __device__ inline uint32_t xchg_offset(const MfmaLayout &l, uint32_t nw) {
    return nw * 4096u <= l.a0 ? 0u : l.total;
}

}  // namespace

// OCC: minimum waves per SIMD the registers are sized for (1: no bound).
// The smallest products (up to 160 limbs) take 4: LDS allows 5 one-wave
// workgroups per SIMD, their per-product phases are latency chains, and the
// unbounded kernel's 180 registers allow only 2.  Larger ones keep the
// compiler's choice.
// KM: every product has 1017-1024 limbs (n32p = 1024, NW = 4) or 505-512
// limbs (n32p = 512, NW = 2) and takes the k-major MFMA order.
// S1: one supertile per wave (every product has at most NW supertiles):
// one row of accumulators, words and carries per wave.
template <int NW, int OCC, class Src, bool KM, bool S1 = false>
__global__ __launch_bounds__(64 * NW, OCC) void bigmul_mfma_kernel(Src src) {
    constexpr int NT = S1 ? 1 : 2;  // rows (supertiles) a wave finalises
    static_assert(!(S1 && KM), "the k-major order takes two supertiles per wave");
    extern __shared__ __align__(16) uint8_t lds[];
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = wave_in_block();
    constexpr uint32_t T = 64 * NW;
    const uint64_t count = src.count();

    Chunks x;
    if (uint64_t(blockIdx.x) < count) fetch_chunks(src.get(blockIdx.x), 64 * wave + lane, x);
    // padded size whose zero pads the LDS holds (nothing else writes them,
    // so they are cleared again only when the layout changes)
    uint32_t pads_for = 0;

    for (uint64_t pair = blockIdx.x; pair < count; pair += gridDim.x) {
        const InstRef in = src.get(pair);
        const uint32_t n32 = in.n, n32p = (n32 + 7) & ~7u;
        const MfmaLayout lo = mfma_layout(n32p, S1 && NW == 1);
        const uint32_t D = lo.D, nb = lo.nb, NE = lo.NE, NBE = lo.NBE, bpad = lo.bpad;
        uint8_t *bpl = lds + lo.bpl;
        uint32_t *summary = reinterpret_cast<uint32_t *>(lds + lo.sum);
        const uint32_t nchunks = n32p / 4;

        // 1. balanced digits: a after kPA zero bytes, b group-reversed into
        //    the two B planes; zero the pads around both.
        uint8_t *adg = lds + lo.a0;
        uint32_t tAB[2];
        recode_chunks<NW>(x, nchunks, summary, tAB);
        const uint32_t tA = tAB[0], tB = tAB[1];
        {
            const uint32_t c = 64 * wave + lane;
            if (c < nchunks) {
                *reinterpret_cast<uint4 *>(adg + kPA + 16 * c) = make_uint4(x.a[0], x.a[1], x.a[2], x.a[3]);
                uint4 v;
                v.x = __builtin_bswap32(x.b[3]);
                v.y = __builtin_bswap32(x.b[2]);
                v.z = __builtin_bswap32(x.b[1]);
                v.w = __builtin_bswap32(x.b[0]);
                *reinterpret_cast<uint4 *>(bpl + (c & 1u) * 16 * NBE + 16 * (bpad + (c >> 1))) = v;
            }
            if (n32p != pads_for) {  // uniform
                pads_for = n32p;
                const uint32_t zlo = kPA / 16, zhi = (lo.A0S - kPA - D) / 16;
                for (uint32_t i = tid; i < zlo + zhi; i += T) {
                    const uint32_t q = i < zlo ? i : (kPA + D) / 16 + (i - zlo);
                    *reinterpret_cast<uint4 *>(adg + 16 * q) = make_uint4(0, 0, 0, 0);
                }
                const uint32_t nz = NBE - nb;
                for (uint32_t i = tid; i < 2 * nz; i += T) {
                    const uint32_t pl = i / nz, e = i - pl * nz;
                    const uint32_t ent = e < bpad ? e : nb + e;
                    *reinterpret_cast<uint4 *>(bpl + pl * 16 * NBE + 16 * ent) = make_uint4(0, 0, 0, 0);
                }
            }
        }
        __syncthreads();

        // 2. the 8-byte windows of a: entry x = digit bytes x - kPA .. x - kPA + 7,
        //    two entries (16 bytes) per thread and step
        {
            const uint32_t *a0w = reinterpret_cast<const uint32_t *>(adg);
            for (uint32_t x2 = tid; 2 * x2 < NE; x2 += T) {
                const uint32_t q = x2 >> 1, sh = 2 * (x2 & 1u);
                const uint32_t w0 = a0w[q], w1 = a0w[q + 1], w2 = a0w[q + 2];
                uint4 v;
                v.x = __builtin_amdgcn_alignbyte(w1, w0, sh);
                v.y = __builtin_amdgcn_alignbyte(w2, w1, sh);
                v.z = __builtin_amdgcn_alignbyte(w1, w0, sh + 1);
                v.w = __builtin_amdgcn_alignbyte(w2, w1, sh + 1);
                *reinterpret_cast<uint4 *>(lds + 16 * x2) = v;
            }
        }
        __syncthreads();

        // next pair's operands, in flight during the products
        if (pair + gridDim.x < count) fetch_chunks(src.get(pair + gridDim.x), 64 * wave + lane, x);

        // 3. MFMA.  Wave role p (rotating with the pair so that every SIMD
        //    sees the light band-edge and heavy middle supertiles) finalises
        //    supertiles s0 = 2 p and s1 = 2 p + 1 (S1: supertile p).
        const uint32_t nst = (n32p + 127) / 128, npt = (nst + NT - 1) / NT;
        const uint32_t r = lane & 31u, g = lane >> 5;
        const uint32_t pw = (wave + uint32_t(pair % NW)) % NW;
        const uint32_t s0 = NT * pw, s1 = s0 + 1;
        const bool has0 = pw < npt, has1 = !S1 && has0 && s1 < nst;
        const uint32_t oA = 8 * (r + kPA - 16 * g - 15);
        uint32_t Lo[2][4] = {}, Hi[2][4] = {};
        // Lo / Hi of supertile st from its coefficient sums acc (plus the
        // word sums ext of the other wave, k-major order)
        auto finalise = [&](const v16i &acc, uint32_t st, const int64_t (&ext)[4], uint32_t (&lo4)[4],
                            uint32_t (&hi4)[4]) {
            // acc[4j + i] at lane (r, g) is coefficient 32 K + 8 j + 4 g + i,
            // K = 32 st + r: the four bytes of word w = 8 K + 2 j + g.
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t w = 256 * st + 8 * r + 2 * uint32_t(j) + g;
                int32_t c[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) c[e] = acc[4 * j + e];
                if (w >= n32p && w < 2 * n32p && (tA | tB)) {
                    const uint32_t m = w - n32p, cc = m >> 2;
                    const uint32_t aw = *reinterpret_cast<const uint32_t *>(adg + kPA + 4 * m);
                    const uint32_t bw = *reinterpret_cast<const uint32_t *>(
                        bpl + (cc & 1u) * 16 * NBE + 16 * (bpad + (cc >> 1)) + 4 * (3 - (m & 3u)));
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        c[e] += int32_t(tA) * sbyte(bw, 3 - e) + int32_t(tB) * sbyte(aw, e);
                }
                uint64_t V = uint64_t(ext[j]) + uint64_t(int64_t(c[0])) + (uint64_t(int64_t(c[1])) << 8) +
                             (uint64_t(int64_t(c[2])) << 16) + (uint64_t(int64_t(c[3])) << 24);
                V += (1ull << 63) - (w > 0 ? (1ull << 31) : 0ull);
                lo4[j] = uint32_t(V);
                hi4[j] = uint32_t(V >> 32);
            }
        };
        if constexpr (KM) {
            // group pw / 2 = supertiles 4 (pw / 2) + i, residues of parity
            // pw % 2; all eight supertiles exist (has0 = has1 = true)
            static_assert(NW == 2 || NW == 4, "the k-major order takes two or four waves");
            const uint32_t grp = pw >> 1, q = pw & 1u;
            const uint8_t *bbs = bpl + g * 16 * NBE + 16 * (32 * 4 * grp + r + bpad);
            v16i acc[4] = {};
            if constexpr (NW == 2) {
                if (q == 0) mfma_kmajor_512<0>(lds, oA, bbs, 0, acc);
                else mfma_kmajor_512<2>(lds, oA, bbs, 1, acc);
            } else if (grp == 0) {
                if (q == 0) mfma_kmajor_1024<false, 0>(lds, oA, bbs, 0, acc);
                else mfma_kmajor_1024<false, 2>(lds, oA, bbs, 1, acc);
            } else {
                if (q == 0) mfma_kmajor_1024<true, 0>(lds, oA, bbs, 1, acc);
                else mfma_kmajor_1024<true, 2>(lds, oA, bbs, 2, acc);
            }
            __syncthreads();  // every wave is done with the windows of a
            int64_t *xb = reinterpret_cast<int64_t *>(lds + xchg_offset(lo, NW));
            // slot (pw, t, j): the sender's partial sums of word j of the
            // receiver's supertile t, 64 lanes of 8 bytes
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int j = 0; j < 4; ++j) xb[((pw * 2 + t) * 4 + j) * 64 + lane] = word_sum(acc[2 + t], j);
            __syncthreads();
            const uint32_t peer = pw ^ 1u;
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                int64_t ext[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) ext[j] = xb[((peer * 2 + t) * 4 + j) * 64 + lane];
                finalise(acc[t], s0 + uint32_t(t), ext, Lo[t], Hi[t]);
            }
        } else {
            if (has0) {
                const uint8_t *bb0 = bpl + g * 16 * NBE + 16 * (32 * s0 + r + bpad);
                const uint8_t *bb1 = bb0 + 16 * 32;
                const int32_t lo0 = max(0, int32_t(32 * s0) - int32_t(nb) + 1);
                const int32_t hi0 = min(int32_t(nb), int32_t(32 * s0 + 31)) + 1;
                const int32_t lo1 = has1 ? max(0, int32_t(32 * s1) - int32_t(nb) + 1) : hi0;
                const int32_t hi1 = has1 ? min(int32_t(nb), int32_t(32 * s1 + 31)) + 1 : hi0;
                v16i acc[2] = {};
                if constexpr (S1) {
                    // one supertile, whose band is never empty (32 s0 < 2 nb):
                    // its first step starts the accumulator
                    acc[0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(
                        load_a_plain(lds, oA, lo0), *reinterpret_cast<const v4i *>(bb0 - 16 * lo0), v16i{}, 0, 0, 0);
                    mfma_steps<1, true>(lo0 + 1, hi0, lds, oA, bb0, bb1, acc);
                } else {
                    mfma_steps<1>(lo0, min(lo1, hi0), lds, oA, bb0, bb1, acc);
                }
                if (has1) {
                    mfma_steps<3>(lo1, hi0, lds, oA, bb0, bb1, acc);
                    mfma_steps<2>(max(hi0, lo1), hi1, lds, oA, bb0, bb1, acc);
                }
                const int64_t none[4] = {};
#pragma unroll
                for (int t = 0; t < NT; ++t) finalise(acc[t], s0 + uint32_t(t), none, Lo[t], Hi[t]);
            }
        }
        // 4. product = L + H in registers.  Lane (r, g) holds the low and
        //    high words of V_w for w = 256 st + 8 r + 2 j + g; two lane swaps
        //    (r, 0) <-> (r, 1) give it words 8 r + 4 g + 0..3 of supertile
        //    st, chunk 2 r + g of row st of the product, whose high addends
        //    are the high words of the word below each.  Wave pw owns rows
        //    s0, s1 (absent rows, and words at or above 2 n32p, lie above
        //    every stored word and only carry upwards).
        uint32_t x[2][4], hv[2][4], y[2][4];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const auto l02 = __builtin_amdgcn_permlane32_swap(Lo[t][0], Lo[t][2], false, false);
            const auto l13 = __builtin_amdgcn_permlane32_swap(Lo[t][1], Lo[t][3], false, false);
            const auto h02 = __builtin_amdgcn_permlane32_swap(Hi[t][0], Hi[t][2], false, false);
            const auto h13 = __builtin_amdgcn_permlane32_swap(Hi[t][1], Hi[t][3], false, false);
            x[t][0] = l02[0]; x[t][1] = l02[1]; x[t][2] = l13[0]; x[t][3] = l13[1];
            hv[t][0] = h02[0]; hv[t][1] = h02[1]; hv[t][2] = h13[0]; hv[t][3] = h13[1];
        }
        // the word below chunk 2 r + g: chunk 2 r + g - 1, at lane r (g = 1)
        // or r - 1 + 32 (g = 0); below row st's chunk 0, the last word of
        // row st - 1 (the other row of this wave, or the wave below's, passed
        // in the recode summary words, dead by now)
        uint32_t *bnd = summary;
        if constexpr (NW > 1)
            if (lane == 0) bnd[pw] = __builtin_amdgcn_readlane(hv[NT - 1][3], 63);
        const int src = int(g ? lane - 32 : lane + 31);
        uint32_t below[2];
#pragma unroll
        for (int t = 0; t < NT; ++t) below[t] = __shfl(hv[t][3], src);
        if constexpr (NW > 1) __syncthreads();
        if (lane == 0) {
            below[0] = pw > 0 ? bnd[pw - 1] : 0u;
            if constexpr (NT > 1) below[1] = __builtin_amdgcn_readlane(hv[0][3], 63);
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            y[t][0] = below[t];
            y[t][1] = hv[t][0];
            y[t][2] = hv[t][1];
            y[t][3] = hv[t][2];
        }
        // carry scan over the wave's two rows in chunk order, then over the
        // waves (rows 2 pw, 2 pw + 1 lie above those of waves < pw)
        const uint32_t cpos = 2 * r + g;
        uint32_t sm[2][4];
        uint64_t G[2], Pm[2];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const uint32_t gc = add_words<4>(x[t], y[t], sm[t]);
            G[t] = lanes_to_chunks(ballot(gc != 0));
            Pm[t] = lanes_to_chunks(ballot(all_ones<4>(sm[t])));
        }
        uint32_t cin = 0, allp = 1;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            cin = wave_carry(G[t], Pm[t], cin).out;
            allp &= Pm[t] == ~0ull ? 1u : 0u;
        }
        uint32_t *csum = summary + 8;
        if constexpr (NW > 1) {
            if (lane == 0) csum[pw] = cin | (allp << 1);
            __syncthreads();
        }
        cin = 0;
        for (uint32_t v = 0; v < pw; ++v) {
            const uint32_t sv = csum[v];
            cin = (sv & 1u) | ((sv >> 1) & cin);
        }
        const GlobalSink sink{in.c, 2 * n32, (reinterpret_cast<uintptr_t>(in.c) & 15) == 0};
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const WaveCarry wc = wave_carry(G[t], Pm[t], cin);
            add_carry_words<4>(sm[t], uint32_t(wc.into >> cpos) & 1u);
            cin = wc.out;
            const uint32_t c = 64 * (s0 + uint32_t(t)) + cpos;
            if ((t == 0 ? has0 : has1) && 4 * c < 2 * n32) sink(c, sm[t]);
        }
        __syncthreads();  // the summary words are free for the next pair
    }
}

uint32_t mfma_max_limbs() { return 1024; }

// Waves per workgroup: one per pair of supertiles (1024 output digits each).
static uint32_t mfma_waves(uint32_t nmax) {
    const uint32_t n32p = (nmax + 7) & ~7u;
    const uint32_t nst = (n32p + 127) / 128, h = (nst + 1) / 2;
    return h <= 1 ? 1 : h <= 2 ? 2 : 4;
}

// Dynamic LDS bytes of a launch whose products have at most nmax limbs:
// the largest layout, with the partial-sum exchange where it lies past it.
template <int NW, bool KM, bool S1 = false>
static uint32_t mfma_lds_bytes(uint32_t nmax) {
    const MfmaLayout l = mfma_layout((nmax + 7) & ~7u, S1 && NW == 1);
    return KM ? std::max(l.total, xchg_offset(l, NW) + NW * 4096u) : l.total;
}

template <int NW, int OCC, class Src, bool KM = false, bool S1 = false>
static hipError_t launch_nw(const Src &src, uint32_t nmax, uint64_t count, hipStream_t st, int num_cus) {
    const uint32_t lds_bytes = mfma_lds_bytes<NW, KM, S1>(nmax);
    const void *fn = reinterpret_cast<const void *>(&bigmul_mfma_kernel<NW, OCC, Src, KM, S1>);
    // (LDS bytes << 32 | resident workgroups per CU) of the last launch shape
    static std::atomic<uint64_t> occ{0}, lds_set{0};
    hipError_t e = lds_limit_once(fn, lds_set);
    if (e != hipSuccess) return e;
    uint64_t o = occ.load(std::memory_order_relaxed);
    if ((o >> 32) != lds_bytes) {
        int nblk = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nblk, fn, 64 * NW, lds_bytes);
        if (e != hipSuccess) return e;
        o = (uint64_t(lds_bytes) << 32) | uint32_t(nblk < 1 ? 1 : nblk);
        occ.store(o, std::memory_order_relaxed);
    }
    // persistent workgroups: each loops over pairs, prefetching the next
    const uint64_t cap = uint64_t(uint32_t(o)) * uint64_t(num_cus > 0 ? num_cus : 1);
    const uint32_t grid = uint32_t(count < cap ? count : cap);
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL((bigmul_mfma_kernel<NW, OCC, Src, KM, S1>), dim3(grid), dim3(64 * NW), lds_bytes, st, src);
    return hipGetLastError();
}

template <class Src>
static hipError_t launch_mfma(const Src &src, uint32_t nmax, uint64_t count, hipStream_t st, int num_cus) {
    if (nmax > mfma_max_limbs()) return hipErrorInvalidValue;
    switch (mfma_waves(nmax)) {
        case 1:
            // one-wave workgroups: registers for 4 per SIMD when LDS holds 16
            // per CU (3, sized the same way at 2^13 bits, measured slower)
            if (mfma_layout((nmax + 7) & ~7u).total * 16 <= 160 * 1024)
                return ((nmax + 7) & ~7u) <= 128 ? launch_nw<1, 4, Src, false, true>(src, nmax, count, st, num_cus)
                                                 : launch_nw<1, 4>(src, nmax, count, st, num_cus);
            return launch_nw<1, 1>(src, nmax, count, st, num_cus);
        case 2: return launch_nw<2, 1>(src, nmax, count, st, num_cus);
        default: return launch_nw<4, 1>(src, nmax, count, st, num_cus);
    }
}

hipError_t launch_bigmul_mfma(const uint32_t *a, const uint32_t *b, uint32_t *c, uint32_t n32, uint64_t batch,
                              hipStream_t st, int num_cus) {
    if (batch == 0) return hipSuccess;
    const UniformInst src{a, b, c, n32, batch};
    // 1017-1024 limbs (eight supertiles, 128 digit blocks) and 505-512 limbs
    // (four supertiles, 64 digit blocks): the k-major order
    if (((n32 + 7) & ~7u) == 1024) return launch_nw<4, 3, UniformInst, true>(src, n32, batch, st, num_cus);
    if (((n32 + 7) & ~7u) == 512) return launch_nw<2, 3, UniformInst, true>(src, n32, batch, st, num_cus);
    return launch_mfma(src, n32, batch, st, num_cus);
}

hipError_t launch_bigmul_mfma_list(const ListInst &src, uint32_t nmax, uint64_t count_max, hipStream_t st,
                                   int num_cus) {
    return launch_mfma(src, nmax, count_max, st, num_cus);
}

}  // namespace bi
