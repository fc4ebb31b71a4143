// Internal (C++) interfaces between the C ABI layer and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/bigint.h"

namespace bi {

struct AddTune {
    uint64_t max_waves = 1u << 16;  // grid cap (waves); kernels grid-stride beyond it
    int rows = 4;                   // rows of 64 chunks each wave loads before consuming (2, 4, 8)
    bool nt = false;                // non-temporal loads and stores
};

// Per-device state owned by a context.
struct Ctx {
    int device = 0;
    int num_cus = 256;
    AddTune add;
};

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

bi_status dispatch_bigmul(Ctx &c, const void *a, const void *b, void *out, uint32_t n32, uint64_t batch, int algo,
                          hipStream_t st);
bi_status dispatch_bigadd_v(Ctx &c, const void *a, const void *b, void *out, uint8_t *carry, const bi_desc *desc,
                            uint64_t count, uint32_t limb_bits, hipStream_t st);
bi_status dispatch_bigmul_v(Ctx &c, const void *a, const void *b, void *out, const bi_desc *desc, uint64_t count,
                            uint32_t limb_bits, int algo, hipStream_t st);

// Sets the calling thread's bi_last_error() message and returns s.
bi_status set_error(bi_status s, const char *fmt, ...);

}  // namespace bi
