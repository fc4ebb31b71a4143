// Multiply-accumulate step of the VALU schoolbook (Section 3.1): a 64-bit
// accumulator plus a 32-bit overflow count per output coefficient.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bi {

// acc += a * b (64-bit), cnt += carry out of that addition: one
// v_mad_u64_u32 (whose carry-out lands in an SGPR pair) and one
// v_addc_co_u32.  The compiler otherwise splits this into a multiply, an add,
// a 64-bit compare and a select.  a is wave-uniform (an SGPR operand).
__device__ __forceinline__ void mac(uint64_t &acc, uint32_t &cnt, uint32_t a, uint32_t b) {
    uint64_t cc, unused;
    asm("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(acc), "=s"(cc) : "s"(a), "v"(b));
    asm("v_addc_co_u32_e64 %0, %1, %0, 0, %2" : "+v"(cnt), "=s"(unused) : "s"(cc));
}

// The same with a per-lane (VGPR) a.
__device__ __forceinline__ void mac_v(uint64_t &acc, uint32_t &cnt, uint32_t a, uint32_t b) {
    uint64_t cc, unused;
    asm("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(acc), "=s"(cc) : "v"(a), "v"(b));
    asm("v_addc_co_u32_e64 %0, %1, %0, 0, %2" : "+v"(cnt), "=s"(unused) : "s"(cc));
}

}  // namespace bi
