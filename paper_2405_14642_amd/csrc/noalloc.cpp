// Fixed device scratch for callers that cannot allocate device memory: one
// file-scope device array per GPU, holding every scratch buffer of
// bigmul_noalloc's kernels.  Its device address is looked up once per device
// at context creation (with that device current) and kept per device; host
// code never passes the array's name itself to a kernel or a copy.
#include <hip/hip_runtime.h>

#include <mutex>

#include "bi_internal.hpp"

namespace bi {

namespace {

__device__ __align__(256) uint8_t scratch[kFixedScratchBytes];

std::mutex g_mu;
void *g_addr[kMaxDevices] = {};  // device address of `scratch` on each device

}  // namespace

bi_status fixed_scratch_init(int device, void **out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return set_error(BI_ENODEV, "device %d beyond %d", device, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(BI_EHIP, "hipGetSymbolAddress of the fixed scratch: %s", hipGetErrorString(e));
        g_addr[device] = p;
    }
    *out = g_addr[device];
    return BI_OK;
}

}  // namespace bi
