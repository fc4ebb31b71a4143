// Context set-up and dispatch from the C ABI to the kernel launchers.
#include <hip/hip_runtime.h>

#include "bi_internal.hpp"

namespace bi {

bi_status ctx_init(Ctx &c, int device, const hipDeviceProp_t &prop) {
    c.device = device;
    c.num_cus = prop.multiProcessorCount;
    c.add.max_waves = uint64_t(prop.multiProcessorCount) * 64;
    return BI_OK;
}

void ctx_release(Ctx &c) { (void)c; }

bi_status dispatch_bigadd_v(Ctx &c, const void *a, const void *b, void *out, uint8_t *carry, const bi_desc *desc,
                            uint64_t count, uint32_t limb_bits, hipStream_t st) {
    hipError_t e = launch_bigadd_ragged(a, b, out, carry, desc, count, limb_bits, st, c.add);
    if (e != hipSuccess) return set_error(BI_EHIP, "bigadd_v launch: %s", hipGetErrorString(e));
    return BI_OK;
}

bi_status dispatch_bigmul(Ctx &c, const void *a, const void *b, void *out, uint32_t n32, uint64_t batch, int algo,
                          hipStream_t st) {
    (void)c; (void)a; (void)b; (void)out; (void)n32; (void)batch; (void)st;
    return set_error(BI_EALGO, "multiplication algorithm %d is not available", algo);
}

bi_status dispatch_bigmul_v(Ctx &c, const void *a, const void *b, void *out, const bi_desc *desc, uint64_t count,
                            uint32_t limb_bits, int algo, hipStream_t st) {
    (void)c; (void)a; (void)b; (void)out; (void)desc; (void)count; (void)limb_bits; (void)st;
    return set_error(BI_EALGO, "multiplication algorithm %d is not available", algo);
}

}  // namespace bi
