// Internal (C++) interfaces between the C ABI layer and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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

struct NttConst {
    uint32_t p[kNttPrimes], pneg[kNttPrimes];     // modulus, -p^-1 mod 2^32
    uint32_t scale[kNttPrimes][kNttLogLmax + 1];  // 2^-l * 2^32 mod p
    uint32_t scale_sh[kNttPrimes][kNttLogLmax + 1];
    uint32_t crt, crt_sh;                         // p1^-1 mod p2 and its Shoup companion
    const uint2 *fwd[kNttPrimes];                 // twiddle blocks (w^e, Shoup), w of order Lmax
    const uint2 *inv[kNttPrimes];                 // the same for w^-1
};

struct NttTables {
    NttConst c{};
    uint2 *dev = nullptr;
};

bi_status ntt_setup(NttTables &t);
void ntt_release(NttTables &t);
bi_status field_info(uint64_t p, bi_ntt_field_info *out);

// Device scratch owned by a context (grown on demand).
struct Scratch {
    void *ptr = nullptr;
    size_t bytes = 0;
};

// Per-device state owned by a context.
struct Ctx {
    int device = 0;
    int num_cus = 256;
    AddTune add;
    NttTables ntt;
    Scratch scratch;
};

// Returns a device buffer of at least `bytes` owned by the context; growing it
// synchronises `st` first so no queued kernel still uses the old buffer.
bi_status ctx_scratch(Ctx &c, size_t bytes, hipStream_t st, void **out);

bi_status ctx_init(Ctx &c, int device, const hipDeviceProp_t &prop);
void ctx_release(Ctx &c);

// out = a + b over `batch` instances of `inst_bytes` bytes each (a multiple of 4).
hipError_t launch_bigadd(const void *a, const void *b, void *out, uint8_t *carry, uint64_t inst_bytes,
                         uint64_t batch, hipStream_t st, const AddTune &t);
hipError_t launch_bigadd_ragged(const void *a, const void *b, void *out, uint8_t *carry, const bi_desc *desc,
                                uint64_t count, uint32_t limb_bits, hipStream_t st, const AddTune &t);

struct ValuPlan {
    int Q = 2;       // output coefficients per lane
    int NW = 1;      // waves per workgroup
    size_t lds = 0;  // dynamic LDS bytes
};
ValuPlan valu_plan(uint32_t n);
hipError_t launch_bigmul_valu(const uint32_t *a, const uint32_t *b, uint32_t *c, uint32_t n, uint64_t batch,
                              hipStream_t st, int num_cus);

// NTT multiplication of n32-limb operands: the four transforms of every pair
// (2 operands x 2 primes, L words each) go to the scratch `tr`
// (ntt_scratch_bytes), then CRT and carry produce the product.
uint32_t ntt_log_len(uint32_t n32);  // log2 of the transform length, 0 if too large
size_t ntt_scratch_bytes(uint32_t n32, uint64_t batch);
hipError_t launch_bigmul_ntt(const NttConst &k, const uint32_t *a, const uint32_t *b, uint32_t *c, uint32_t n32,
                             uint64_t batch, uint32_t *tr, hipStream_t st);

// int8-MFMA schoolbook for up to mfma_max_limbs() 32-bit limbs.
uint32_t mfma_max_limbs();
hipError_t launch_bigmul_mfma(const uint32_t *a, const uint32_t *b, uint32_t *c, uint32_t n32, uint64_t batch,
                              hipStream_t st);

bi_status dispatch_bigmul(Ctx &c, const void *a, const void *b, void *out, uint32_t n32, uint64_t batch, int algo,
                          hipStream_t st);
bi_status dispatch_bigadd_v(Ctx &c, const void *a, const void *b, void *out, uint8_t *carry, const bi_desc *desc,
                            uint64_t count, uint32_t limb_bits, hipStream_t st);
bi_status dispatch_bigmul_v(Ctx &c, const void *a, const void *b, void *out, const bi_desc *desc, uint64_t count,
                            uint32_t limb_bits, int algo, hipStream_t st);

// Sets the calling thread's bi_last_error() message and returns s.
bi_status set_error(bi_status s, const char *fmt, ...);

}  // namespace bi
