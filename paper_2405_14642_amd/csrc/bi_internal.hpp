// Internal (C++) interfaces between the C ABI layer and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

#include "../../include/bigint.h"

namespace bi {

struct AddTune {
    uint64_t max_waves = 1u << 16;  // grid cap (waves); kernels grid-stride beyond it
    int rows = 4;                   // rows of 64 chunks each wave loads before consuming (2, 4, 8)
    bool nt = true;                 // non-temporal loads and stores
    // Instances of 2 / 3-4 / 5-8 rows: barrier-free one-wave-per-instance
    // schedule instead of the workgroup-cooperative one.
    bool multi2 = false, multi4 = false, multi8 = false;
};

constexpr uint32_t kMaxLimbs32 = BI_MAX_BITS / 32;  // 8192
constexpr uint32_t kNumClasses = 10;               // ragged size classes: <= 16, 32, ..., 8192 limbs
uint32_t class_nmax(uint32_t c);

// Per-context tuning: multiplication algorithm per size class for uniform
// batches (BI_MUL_AUTO in bigmul) and for ragged ones (bigmul_v and the
// stream queue, whose instances spread over the class's sizes).
struct Tune {
    int mul_algo[kNumClasses];
    int list_algo[kNumClasses];
    // VALU schoolbook schedule per class: output words per lane (Q = 2 or 4)
    // and waves per workgroup; 0 = the size rule of valu_plan.
    uint8_t valu_q[kNumClasses];
    uint8_t valu_nw[kNumClasses];
    // Karatsuba: levels stop at base products of at most kara_base[k] words
    uint16_t kara_base[kNumClasses];
};
bool algo_supports(int algo, uint32_t n32);
// The algorithm bigmul runs for `algo` at n32 words: BI_MUL_AUTO resolves to
// the size class's tuned choice (the VALU schoolbook if that cannot run n32).
int resolve_algo(const Tune &tune, uint32_t n32, int algo);

// NTT field constants (two primes below 2^31) and device twiddle tables.
constexpr int kNttPrimes = 2;
constexpr int kNttLogLmax = 15;                  // transforms of up to 2^15 points
constexpr int kNttLogLmin = 11;                  // and at least 2^11 (64 threads)
constexpr uint32_t kNttLmax = 1u << kNttLogLmax;
// Per prime and direction the twiddle block holds: [0, Lmax) w^e;
// [kNttT1, +1024) the pass-1 table; from ntt_t0_offset(M) the pass-0 table of
// length 2^M.
constexpr uint32_t kNttT1 = kNttLmax;
__host__ __device__ constexpr uint32_t ntt_t0_offset(uint32_t m) {
    return kNttT1 + 1024 + ((1u << m) - (1u << kNttLogLmin));
}
constexpr uint32_t kNttTableWords = ntt_t0_offset(kNttLogLmax + 1);

// Output scales 2^-l 2^32 are kept up to l = kNttScaleMax: a row transform of
// up to 2^15 points times a column transform of up to 2^7 (products beyond
// 2^18 bits, as a two-dimensional convolution).
constexpr int kNttScaleMax = kNttLogLmax + 7;

struct NttConst {
    uint32_t p[kNttPrimes], pneg[kNttPrimes];     // modulus, -p^-1 mod 2^32
    uint32_t one_sh[kNttPrimes];                  // Shoup companion of 1: floor(2^32 / p)
    uint32_t scale[kNttPrimes][kNttScaleMax + 1];  // 2^-l * 2^32 mod p
    uint32_t scale_sh[kNttPrimes][kNttScaleMax + 1];
    uint32_t crt, crt_sh;                         // p1^-1 mod p2 and its Shoup companion
    const uint2 *fwd[kNttPrimes];                 // twiddle blocks (w^e, Shoup), w of order Lmax
    const uint2 *inv[kNttPrimes];                 // the same for w^-1
};

// PrimeField64 of Section 4.1: p = 29 2^57 + 1 (k = 29, n = 57), one prime
// whose 2^61.86 exceeds every product coefficient (< 2^46), so no CRT.  A
// product of operands with up to H coefficients is split into its cyclic and
// negacyclic convolutions of length H (half the zero-padded length), which
// give the low and high halves of the coefficient vector.  Residues are
// 64-bit; twiddles are stored in Montgomery form (w 2^64 mod p).
constexpr uint64_t kP64 = 4179340454199820289ull;  // 29 * 2^57 + 1
constexpr int kP64LogHmax = 14;                    // half-length transforms of up to 2^14 points
constexpr int kP64LogHmin = 11;
constexpr uint32_t kP64Hmax = 1u << kP64LogHmax;
// Twiddle block per direction, as for the two-prime tables: [0, Hmax) w^e;
// [kP64T1, +1024) the pass-1 table; from p64_t0_offset(M) the pass-0 table.
constexpr uint32_t kP64T1 = kP64Hmax;
__host__ __device__ constexpr uint32_t p64_t0_offset(uint32_t m) {
    return kP64T1 + 1024 + ((1u << m) - (1u << kP64LogHmin));
}
constexpr uint32_t kP64TableWords = p64_t0_offset(kP64LogHmax + 1);

struct NttConst64 {
    uint64_t scale[kP64LogHmax + 1];  // Montgomery form of 2^-l 2^64 (undoes the pointwise R^-1)
    const uint64_t *fwd, *inv;        // twiddle blocks, w of order Hmax
    const uint64_t *twist, *untwist;  // psi^e and psi^-e for e < Hmax, psi of order 2 Hmax
};

struct NttTables {
    NttConst c{};
    uint2 *dev = nullptr;
    NttConst64 c64{};
    uint64_t *dev64 = nullptr;
};

bi_status ntt_setup(NttTables &t);
bi_status ntt64_setup(NttTables &t);
void ntt_release(NttTables &t);
bi_status field_info(uint64_t p, bi_ntt_field_info *out);

// Device scratch owned by a context (grown on demand).
struct Scratch {
    void *ptr = nullptr;
    size_t bytes = 0;
};

// Where the instances of a launch come from.  Uniform: pair p at a + p n.
// List: entry p of a size-class list of ragged descriptors (bigmul_v).
struct InstRef {
    const uint32_t *a, *b;
    uint32_t *c;
    uint32_t n;  // 32-bit limbs
};

struct UniformInst {
    const uint32_t *a, *b;
    uint32_t *c;
    uint32_t n;
    uint64_t batch;
    __device__ __forceinline__ uint64_t count() const { return batch; }
    __device__ __forceinline__ InstRef get(uint64_t p) const {
        return InstRef{a + p * n, b + p * n, c + p * 2 * n, n};
    }
};

// Block q < k of ONE long operand pair cut into blocks of bw words: words
// [q bw, min((q + 1) bw, n32)) of a and b (the last block may be shorter).
struct BlockInst {
    const uint32_t *a, *b;
    uint64_t n32;
    uint32_t bw, k;
    __device__ __forceinline__ uint64_t count() const { return k; }
    __device__ __forceinline__ InstRef get(uint64_t q) const {
        const uint64_t off = q * bw, rem = n32 - off;
        return InstRef{a + off, b + off, nullptr, uint32_t(rem < bw ? rem : bw)};
    }
};

struct ListInst {
    const uint32_t *a, *b;
    uint32_t *c;
    const bi_desc *desc;
    const uint32_t *list;   // descriptor indices of this size class
    const uint32_t *count_ptr;
    uint32_t words_per_limb;  // 1 (32-bit limbs) or 2 (64-bit limbs)
    __device__ __forceinline__ uint64_t count() const { return *count_ptr; }
    __device__ __forceinline__ InstRef get(uint64_t p) const {
        const bi_desc d = desc[list[p]];
        const uint32_t w = words_per_limb;
        return InstRef{a + d.a_off * w, b + d.b_off * w, c + d.out_off * w, d.n_limbs * w};
    }
};

// Per-device state owned by a context.
struct Ctx {
    int device = 0;
    int num_cus = 256;
    AddTune add;
    Tune tune{};
    NttTables ntt;
    Scratch scratch;
    char arch[64] = {};               // gcnArchName of the device
    int hip_version = 0;              // hipRuntimeGetVersion
    void *fixed_scratch = nullptr;    // this device's fixed scratch array (bigmul_noalloc)
};

// The fixed scratch array of bigmul_noalloc: kFixedScratchBytes of device
// memory per GPU, part of the library's code object.  fixed_scratch_init
// (with `device` current) returns its device address on that device, looked
// up once per device.
constexpr size_t kFixedScratchBytes = size_t(BI_NOALLOC_SCRATCH_BYTES);
constexpr int kMaxDevices = 64;
bi_status fixed_scratch_init(int device, void **out);


// Returns a device buffer of at least `bytes` owned by the context; growing it
// synchronises the device first so no queued kernel still uses the old buffer.
bi_status ctx_scratch(Ctx &c, size_t bytes, hipStream_t st, void **out);

bi_status ctx_init(Ctx &c, int device, const hipDeviceProp_t &prop);
void ctx_release(Ctx &c);

// out = a + b over `batch` instances of `inst_bytes` bytes each (a multiple of 4).
hipError_t launch_bigadd(const void *a, const void *b, void *out, uint8_t *carry, uint64_t inst_bytes,
                         uint64_t batch, hipStream_t st, const AddTune &t);
// Addition of one integer of n32 32-bit words across workgroups; scratch
// holds large_add_scratch_bytes(large_add_tiles(n32, large_add_chunk_words(a,
// b, out))) bytes, 16-byte aligned.
int large_add_chunk_words(const void *a, const void *b, const void *out);
uint64_t large_add_tiles(uint64_t n32, int w);
size_t large_add_scratch_bytes(uint64_t tiles);
hipError_t launch_bigadd_large(const void *a, const void *b, void *out, uint8_t *carry, uint64_t n32,
                               uint8_t *scratch, hipStream_t st, int num_cus);
hipError_t launch_bigadd_ragged(const void *a, const void *b, void *out, uint8_t *carry, const bi_desc *desc,
                                uint64_t count, uint32_t limb_bits, hipStream_t st, const AddTune &t);

struct ValuPlan {
    int Q = 2;       // output coefficients per lane
    int NW = 1;      // waves per workgroup
    size_t lds = 0;  // dynamic LDS bytes
};
ValuPlan valu_plan(uint32_t n);                                // the size rule
bool valu_plan_fits(uint32_t n, int Q, int NW, ValuPlan *out);   // LDS of (Q, NW) for n fits a CU
ValuPlan valu_plan_tuned(uint32_t n, const Tune &t);             // the class's tuned plan, else the rule
uint32_t size_class_host(uint32_t n32);
hipError_t launch_bigmul_valu(const uint32_t *a, const uint32_t *b, uint32_t *c, uint32_t n, uint64_t batch,
                              const ValuPlan &p, hipStream_t st, int num_cus);

// NTT multiplication of n32-limb operands: the four transforms of every pair
// (2 operands x 2 primes, L words each) go to the scratch `tr`
// (ntt_scratch_bytes), then CRT and carry produce the product.
uint32_t ntt_log_len(uint32_t n32);  // log2 of the transform length, 0 if too large
size_t ntt_scratch_bytes(uint32_t n32, uint64_t batch);
// `round` bounds the products whose transforms are in tr at once (the batch
// runs in rounds of that many).
hipError_t launch_bigmul_ntt(const NttConst &k, const uint32_t *a, const uint32_t *b, uint32_t *c, uint32_t n32,
                             uint64_t batch, uint32_t *tr, hipStream_t st, uint64_t round, int num_cus);

// Ragged (descriptor-list) launches of one size class; nmax bounds the
// class's limb counts, count_max bounds the class size (the true size is read
// on the device).
hipError_t launch_bigmul_valu_list(const ListInst &src, uint32_t nmax, uint64_t count_max, const ValuPlan &p,
                                   hipStream_t st, int num_cus);
hipError_t launch_bigmul_mfma_list(const ListInst &src, uint32_t nmax, uint64_t count_max, hipStream_t st,
                                   int num_cus);
hipError_t launch_bigmul_ntt_list(const NttConst &K, const ListInst &src, uint32_t nmax, uint64_t count_max,
                                  uint32_t *scratch, hipStream_t st, int num_cus);
// Ragged NTT classes run in rounds of at most kNttListChunk instances of the
// longest transform (more at shorter lengths); scratch for `count` instances.
constexpr uint64_t kNttListChunk = 1024;
size_t ntt_list_scratch_bytes(uint64_t count);

// PrimeField64 NTT multiplication: four half-length transforms per pair (2
// operands x cyclic / negacyclic, H 64-bit words each) in the scratch `tr`
// (ntt64_scratch_bytes), then the halves are recombined and carried.
uint32_t ntt64_log_len(uint32_t n32);  // log2 H, 0 if too large
size_t ntt64_scratch_bytes(uint32_t n32, uint64_t batch);
hipError_t launch_bigmul_ntt64(const NttConst64 &k, const uint32_t *a, const uint32_t *b, uint32_t *c, uint32_t n32,
                               uint64_t batch, uint64_t *tr, hipStream_t st, uint64_t round);
hipError_t launch_bigmul_ntt64_list(const NttConst64 &K, const ListInst &src, uint32_t nmax, uint64_t count_max,
                                    uint64_t *scratch, hipStream_t st, int num_cus);
size_t ntt64_list_scratch_bytes(uint64_t count);

// int8-MFMA schoolbook: one workgroup per product up to mfma_max_limbs()
// 32-bit limbs; above that (up to kMaxLimbs32) the three-kernel large-product
// path, with a scratch slot of mfma_big_slot_bytes(n) per product.
uint32_t mfma_max_limbs();
size_t mfma_big_slot_bytes(uint32_t nmax);
hipError_t launch_bigmul_mfma_big(const uint32_t *a, const uint32_t *b, uint32_t *c, uint32_t n32, uint64_t batch,
                                  uint8_t *scr, hipStream_t st, int num_cus, uint64_t round);
hipError_t launch_bigmul_mfma_big_list(const ListInst &src, uint32_t nmax, uint64_t count_max, uint8_t *scr,
                                       size_t scr_bytes, hipStream_t st, int num_cus);
hipError_t launch_bigmul_mfma(const uint32_t *a, const uint32_t *b, uint32_t *c, uint32_t n32, uint64_t batch,
                              hipStream_t st, int num_cus);

// Fused programs (BI_PROG_*), one workgroup per instance of n32 words.
size_t fused_lds_bytes(int program, uint32_t n32);
hipError_t launch_fused(int program, const uint32_t *a, const uint32_t *b, uint32_t *c, uint32_t n32, uint64_t batch,
                        hipStream_t st, int num_cus);

// Full products of a uniform batch.  Scratch-using algorithms take the
// context's growable buffer, or with `fixed` set that buffer of fixed_bytes
// (never grown: the batch runs in rounds that fit it; BI_ESIZE if one product
// does not).
bi_status dispatch_bigmul(Ctx &c, const void *a, const void *b, void *out, uint32_t n32, uint64_t batch, int algo,
                          hipStream_t st, void *fixed = nullptr, size_t fixed_bytes = 0);
bi_status dispatch_bigadd_v(Ctx &c, const void *a, const void *b, void *out, uint8_t *carry, const bi_desc *desc,
                            uint64_t count, uint32_t limb_bits, hipStream_t st);
// Ragged multiplication core: binning plus one list launch per size class.
// `scratch` holds batch_scratch_bytes(count_max) bytes; the descriptor count
// is count_max, or read on the device from *count_ptr when it is set (so the
// launch sequence can be captured once and replayed with other counts).
size_t batch_scratch_bytes(uint64_t count, int num_cus);
hipError_t launch_bigmul_v_core(const Ctx &c, const Tune &tune, const void *a, const void *b, void *out,
                                const bi_desc *desc, uint64_t count_max, const uint64_t *count_ptr,
                                uint32_t limb_bits, int algo, void *scratch, hipStream_t st);
// The same with the binning done on the host: class k's descriptor indices are
// the host_counts[k] entries of `lists` after those of classes 0..k-1, and
// counts (device) holds the same counts.  Classes with no instance launch
// nothing; the others get grids sized to their count.  scratch holds
// batch_scratch_bytes(max count) bytes.
hipError_t launch_bigmul_v_binned(const Ctx &c, const Tune &tune, const void *a, const void *b, void *out,
                                  const bi_desc *desc, const uint32_t *lists, const uint32_t *counts,
                                  const uint32_t *host_counts, uint32_t limb_bits, int algo, void *scratch,
                                  hipStream_t st);
// Full product of one pair of n32 > 0 words through k^2 block products of bw
// words (2048, 4096 or 8192); scratch holds large_mul_scratch_bytes(n32, bw,
// num_cus) bytes, 256-byte aligned.
size_t large_mul_scratch_bytes(uint64_t n32, uint32_t bw, int num_cus);
hipError_t launch_bigmul_large(const Ctx &c, const uint32_t *a, const uint32_t *b, uint32_t *out, uint64_t n32,
                               uint32_t bw, int algo, uint8_t *scratch, hipStream_t st);
// Block size (words) of bigmul_large's block products for n32-word operands
// when the caller leaves it to the library.
uint32_t large_mul_auto_block(uint64_t n32);

// The same product as a two-dimensional NTT convolution (rows: the k <= 64
// blocks of bw words, 512 <= bw <= 8192, transformed along each block;
// columns: transformed across blocks), then CRT, a fold into words and the
// multi-workgroup addition.  scratch holds large_ntt_scratch_bytes(n32, bw)
// bytes, 256-byte aligned.
constexpr uint32_t kLargeNttMaxBlocks = 64;
uint32_t large_ntt_auto_block(uint64_t n32);
size_t large_ntt_scratch_bytes(uint64_t n32, uint32_t bw);
hipError_t launch_bigmul_large_ntt(const Ctx &c, const uint32_t *a, const uint32_t *b, uint32_t *out, uint64_t n32,
                                   uint32_t bw, uint8_t *scratch, hipStream_t st);
// Ragged list launch of one resolved algorithm `alg` (not BI_MUL_AUTO) over
// instances of up to nmax words; scr holds scr_bytes of scratch, at least
// list_algo_scratch_bytes(alg, nmax, count_max).
size_t list_algo_scratch_bytes(int alg, uint32_t nmax, uint64_t count);
hipError_t launch_bigmul_list_algo(const Ctx &c, const Tune &tune, const ListInst &src, uint32_t nmax,
                                   uint64_t count_max, int alg, void *scr, size_t scr_bytes, hipStream_t st);

// Karatsuba levels over a batched base product.  kara_plan(n, base): operand
// words h[j] of level j (h[0] = n; h[j+1] = ceil(h[j] / 2) rounded up to a
// multiple of 4) down to the first level of at most `base` words (at least
// one level).  The base algorithm is the tuned one of the last level's size
// class (the MFMA schoolbook if that is Karatsuba itself).
constexpr int kKaraMaxLevels = 4;
constexpr uint32_t kKaraBase = 1024;       // default base: products of at most 2^15 bits
constexpr uint32_t kKaraBases[] = {512, 1024, 2048};  // the base sizes tuning chooses from
inline bool kara_base_valid(uint32_t b) {
    for (uint32_t v : kKaraBases)
        if (b == v) return true;
    return false;
}
constexpr uint64_t kKaraListRound = 1024;  // ragged instances per round of levels
constexpr size_t kKaraScratchBudget = size_t(256) << 20;  // uniform batches: scratch per round
struct KaraPlan {
    int levels = 0;
    uint32_t h[kKaraMaxLevels + 1] = {};
};
KaraPlan kara_plan(uint32_t n32, uint32_t base);
// The plan of the size class of n32 words under `tune`.
KaraPlan kara_plan_tuned(const Tune &tune, uint32_t n32);
int kara_base_algo(const Tune &tune, uint32_t h, bool ragged = false);
// Scratch of one round of R top-level instances (list: ragged rounds, which
// also publish the base products as a descriptor list), plus base_bytes for
// the base algorithm.
size_t kara_round_bytes(const KaraPlan &p, uint64_t R, bool list, size_t base_bytes);
// Uniform batch in rounds of `round` instances, each round's levels in `scr`
// (kara_round_bytes(p, round, false, base_bytes) bytes); base_bytes > 0 gives
// the base algorithm that fixed share of the scratch.
bi_status launch_bigmul_kara(Ctx &c, const uint32_t *a, const uint32_t *b, uint32_t *out, uint32_t n32,
                             uint64_t batch, const KaraPlan &p, int base_algo, size_t base_bytes, uint8_t *scr,
                             uint64_t round, hipStream_t st);
// Ragged size-class list of instances of up to nmax words, in rounds that fit
// scr_bytes; kara_list_scratch_bound(count) bytes suffice for every class.
hipError_t launch_bigmul_kara_list(const Ctx &c, const Tune &tune, const ListInst &src, uint32_t nmax,
                                   uint64_t count_max, uint8_t *scr, size_t scr_bytes, hipStream_t st);
size_t kara_list_scratch_bound(uint64_t count);
// Scratch bytes per product of a uniform batch of n32-word products (0 when
// the algorithm needs none).
size_t uniform_algo_scratch_bytes(int alg, uint32_t n32);

bi_status dispatch_bigmul_v(Ctx &c, const void *a, const void *b, void *out, const bi_desc *desc, uint64_t count,
                            uint32_t limb_bits, int algo, hipStream_t st);

bi_status autotune(Ctx &c, hipStream_t st, int *algo_out, uint32_t n_out);
// The context's tuning tables to / from a text file keyed by the device
// architecture and the HIP runtime version.
bi_status tune_save(const Ctx &c, const char *path);
bi_status tune_load(Ctx &c, const char *path);

// Raises kernel `fn`'s dynamic-LDS limit to a whole CU (160 KiB) on the
// current device, once per device: `done` holds one bit per device id (ids
// of 64 and above set the attribute on every call).  Thread-safe: a racing
// second caller repeats the idempotent attribute set.
hipError_t lds_limit_once(const void *fn, std::atomic<uint64_t> &done);

// Sets the calling thread's bi_last_error() message and returns s.
bi_status set_error(bi_status s, const char *fmt, ...);

}  // namespace bi

namespace bi {
// Makes `dev` the current device for the scope of a call, restoring the
// caller's device afterwards.
struct DeviceGuard {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit DeviceGuard(int dev) {
        err = hipGetDevice(&prev);
        if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
        else prev = -1;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};
}  // namespace bi

// The opaque context handle of the C ABI.
struct bi_ctx {
    int device = 0;
    bi::Ctx impl;
};
