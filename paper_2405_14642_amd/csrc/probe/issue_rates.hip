// Register-resident issue-rate probe for the instructions the integer-op
// rooflines count (a measurement aid of the benchmark, not part of the
// arithmetic library).  Each lane runs independent dependency chains of one
// instruction, written in inline asm so the compiler neither folds nor
// reorders them; no memory is touched inside the timed loop.  The kernel also
// reads the shader clock counter (s_memtime) against the constant 100 MHz
// counter (s_memrealtime) on one wave, giving the clock the loop ran at.
//
// C entry (loaded by the benchmark with ctypes):
//   int bi_probe_rate(int kind, int iters, int waves_per_simd,
//                     double *ops_per_s, double *clock_hz, double *seconds);
// kind: 0 v_add_u32, 1 v_addc_co_u32 (VOP3, carry in/out in SGPR pairs),
// 2 v_mad_u64_u32, 3 v_mul_lo_u32, 4 v_mul_hi_u32, 5 v_mfma_i32_32x32x32_i8
// (ops_per_s counts int8 multiply-accumulates), 6 the VALU schoolbook term
// (one v_mad_u64_u32 plus one v_addc_co_u32).  Returns 0, or a HIP error code.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kChains = 8;   // independent chains per lane
constexpr int kUnroll = 4;   // chain steps per loop iteration

#define OP8(a, b, c, d, e, f, g, h) a "\n\t" b "\n\t" c "\n\t" d "\n\t" e "\n\t" f "\n\t" g "\n\t" h

template <int KIND>
__global__ __launch_bounds__(256) void probe_kernel(int iters, uint32_t seed, uint32_t *out, uint64_t *clk) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t t0 = 0, r0 = 0;
    if (t == 0) {
        t0 = __builtin_amdgcn_s_memtime();
        r0 = __builtin_amdgcn_s_memrealtime();
    }
    uint32_t acc = 0;
    if constexpr (KIND == 5) {
        typedef int v16i __attribute__((ext_vector_type(16)));
        typedef int v4i __attribute__((ext_vector_type(4)));
        v16i c[4];
        for (int k = 0; k < 4; ++k)
            for (int e = 0; e < 16; ++e) c[k][e] = 0;
        v4i a, b;
        for (int e = 0; e < 4; ++e) {
            a[e] = int(seed * (t + e + 1));
            b[e] = int(seed ^ (t * 7 + e));
        }
        for (int i = 0; i < iters; ++i) {
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
#pragma unroll
                for (int k = 0; k < 4; ++k) c[k] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c[k], 0, 0, 0);
        }
        for (int k = 0; k < 4; ++k)
            for (int e = 0; e < 16; ++e) acc += uint32_t(c[k][e]);
    } else {
        uint32_t x[kChains], y = seed ^ t;
        uint64_t w[kChains], m[kChains];  // m: wave-wide carry masks (SGPR pairs)
        for (int k = 0; k < kChains; ++k) {
            x[k] = seed + t * (k + 3);
            w[k] = uint64_t(x[k]) * 0x9E3779B9u;
            m[k] = uint64_t(seed) << k;
        }
        // one asm block per step holds all eight chains, so the compiler
        // inserts no hazard padding between chains
        for (int i = 0; i < iters; ++i) {
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                if constexpr (KIND == 0) {
                    asm volatile(OP8("v_add_u32 %0, %0, %8", "v_add_u32 %1, %1, %8", "v_add_u32 %2, %2, %8",
                                     "v_add_u32 %3, %3, %8", "v_add_u32 %4, %4, %8", "v_add_u32 %5, %5, %8",
                                     "v_add_u32 %6, %6, %8", "v_add_u32 %7, %7, %8")
                                 : "+v"(x[0]), "+v"(x[1]), "+v"(x[2]), "+v"(x[3]), "+v"(x[4]), "+v"(x[5]),
                                   "+v"(x[6]), "+v"(x[7])
                                 : "v"(y));
                } else if constexpr (KIND == 3) {
                    asm volatile(OP8("v_mul_lo_u32 %0, %0, %8", "v_mul_lo_u32 %1, %1, %8", "v_mul_lo_u32 %2, %2, %8",
                                     "v_mul_lo_u32 %3, %3, %8", "v_mul_lo_u32 %4, %4, %8", "v_mul_lo_u32 %5, %5, %8",
                                     "v_mul_lo_u32 %6, %6, %8", "v_mul_lo_u32 %7, %7, %8")
                                 : "+v"(x[0]), "+v"(x[1]), "+v"(x[2]), "+v"(x[3]), "+v"(x[4]), "+v"(x[5]),
                                   "+v"(x[6]), "+v"(x[7])
                                 : "v"(y));
                } else if constexpr (KIND == 4) {
                    asm volatile(OP8("v_mul_hi_u32 %0, %0, %8", "v_mul_hi_u32 %1, %1, %8", "v_mul_hi_u32 %2, %2, %8",
                                     "v_mul_hi_u32 %3, %3, %8", "v_mul_hi_u32 %4, %4, %8", "v_mul_hi_u32 %5, %5, %8",
                                     "v_mul_hi_u32 %6, %6, %8", "v_mul_hi_u32 %7, %7, %8")
                                 : "+v"(x[0]), "+v"(x[1]), "+v"(x[2]), "+v"(x[3]), "+v"(x[4]), "+v"(x[5]),
                                   "+v"(x[6]), "+v"(x[7])
                                 : "v"(y));
                } else if constexpr (KIND == 1) {
                    asm volatile(OP8("v_addc_co_u32_e64 %0, %8, %0, %16, %8",
                                     "v_addc_co_u32_e64 %1, %9, %1, %16, %9",
                                     "v_addc_co_u32_e64 %2, %10, %2, %16, %10",
                                     "v_addc_co_u32_e64 %3, %11, %3, %16, %11",
                                     "v_addc_co_u32_e64 %4, %12, %4, %16, %12",
                                     "v_addc_co_u32_e64 %5, %13, %5, %16, %13",
                                     "v_addc_co_u32_e64 %6, %14, %6, %16, %14",
                                     "v_addc_co_u32_e64 %7, %15, %7, %16, %15")
                                 : "+v"(x[0]), "+v"(x[1]), "+v"(x[2]), "+v"(x[3]), "+v"(x[4]), "+v"(x[5]),
                                   "+v"(x[6]), "+v"(x[7]), "+s"(m[0]), "+s"(m[1]), "+s"(m[2]), "+s"(m[3]),
                                   "+s"(m[4]), "+s"(m[5]), "+s"(m[6]), "+s"(m[7])
                                 : "v"(y));
                } else if constexpr (KIND == 2) {
                    asm volatile(OP8("v_mad_u64_u32 %0, %8, %9, %10, %0", "v_mad_u64_u32 %1, %8, %9, %10, %1",
                                     "v_mad_u64_u32 %2, %8, %9, %10, %2", "v_mad_u64_u32 %3, %8, %9, %10, %3",
                                     "v_mad_u64_u32 %4, %8, %9, %10, %4", "v_mad_u64_u32 %5, %8, %9, %10, %5",
                                     "v_mad_u64_u32 %6, %8, %9, %10, %6", "v_mad_u64_u32 %7, %8, %9, %10, %7")
                                 : "+v"(w[0]), "+v"(w[1]), "+v"(w[2]), "+v"(w[3]), "+v"(w[4]), "+v"(w[5]),
                                   "+v"(w[6]), "+v"(w[7]), "=&s"(m[0])
                                 : "v"(x[0]), "v"(y));
                } else if constexpr (KIND == 6) {
                    // the schoolbook's term: a 32 x 32 -> 64-bit product added
                    // into a 64-bit accumulator, its carry-out counted
                    asm volatile(OP8("v_mad_u64_u32 %0, %16, %17, %18, %0\n\tv_addc_co_u32_e64 %8, %16, %8, 0, %16",
                                     "v_mad_u64_u32 %1, %16, %17, %18, %1\n\tv_addc_co_u32_e64 %9, %16, %9, 0, %16",
                                     "v_mad_u64_u32 %2, %16, %17, %18, %2\n\tv_addc_co_u32_e64 %10, %16, %10, 0, %16",
                                     "v_mad_u64_u32 %3, %16, %17, %18, %3\n\tv_addc_co_u32_e64 %11, %16, %11, 0, %16",
                                     "v_mad_u64_u32 %4, %16, %17, %18, %4\n\tv_addc_co_u32_e64 %12, %16, %12, 0, %16",
                                     "v_mad_u64_u32 %5, %16, %17, %18, %5\n\tv_addc_co_u32_e64 %13, %16, %13, 0, %16",
                                     "v_mad_u64_u32 %6, %16, %17, %18, %6\n\tv_addc_co_u32_e64 %14, %16, %14, 0, %16",
                                     "v_mad_u64_u32 %7, %16, %17, %18, %7\n\tv_addc_co_u32_e64 %15, %16, %15, 0, %16")
                                 : "+v"(w[0]), "+v"(w[1]), "+v"(w[2]), "+v"(w[3]), "+v"(w[4]), "+v"(w[5]),
                                   "+v"(w[6]), "+v"(w[7]), "+v"(x[0]), "+v"(x[1]), "+v"(x[2]), "+v"(x[3]),
                                   "+v"(x[4]), "+v"(x[5]), "+v"(x[6]), "+v"(x[7]), "=&s"(m[0])
                                 : "v"(y), "v"(seed));
                }
            }
        }
        for (int k = 0; k < kChains; ++k) acc += x[k] + uint32_t(w[k]) + uint32_t(w[k] >> 32) + uint32_t(m[k]);
    }
    out[t] = acc;
    if (t == 0) {
        clk[0] = __builtin_amdgcn_s_memtime() - t0;
        clk[1] = __builtin_amdgcn_s_memrealtime() - r0;
    }
}

template <int KIND>
hipError_t run(int grid, int iters, uint32_t *out, uint64_t *clk, hipStream_t st) {
    hipLaunchKernelGGL((probe_kernel<KIND>), dim3(grid), dim3(256), 0, st, iters, 0x2405u, out, clk);
    return hipGetLastError();
}

}  // namespace

extern "C" int bi_probe_rate(int kind, int iters, int waves_per_simd, double *ops_per_s, double *clock_hz,
                             double *seconds) {
    if (kind < 0 || kind > 6 || iters < 1 || waves_per_simd < 1 || waves_per_simd > 8 || !ops_per_s || !clock_hz ||
        !seconds)
        return int(hipErrorInvalidValue);
    int dev = 0;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return int(e);
    // 256-thread workgroups = one wave per SIMD; waves_per_simd of them per CU
    const int grid = prop.multiProcessorCount * waves_per_simd;
    uint32_t *out = nullptr;
    uint64_t *clk = nullptr;
    if ((e = hipMalloc(&out, size_t(grid) * 256 * sizeof(uint32_t))) != hipSuccess) return int(e);
    if ((e = hipMalloc(&clk, 2 * sizeof(uint64_t))) != hipSuccess) {
        (void)hipFree(out);
        return int(e);
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    auto launch = [&](int it) -> hipError_t {
        switch (kind) {
            case 0: return run<0>(grid, it, out, clk, nullptr);
            case 1: return run<1>(grid, it, out, clk, nullptr);
            case 2: return run<2>(grid, it, out, clk, nullptr);
            case 3: return run<3>(grid, it, out, clk, nullptr);
            case 4: return run<4>(grid, it, out, clk, nullptr);
            case 5: return run<5>(grid, it, out, clk, nullptr);
            default: return run<6>(grid, it, out, clk, nullptr);
        }
    };
    e = launch(iters / 8 + 1);  // warm-up (clock ramp, code load)
    if (e == hipSuccess) e = hipEventRecord(e0, nullptr);
    if (e == hipSuccess) e = launch(iters);
    if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    uint64_t c[2] = {0, 0};
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess) e = hipMemcpy(c, clk, sizeof(c), hipMemcpyDeviceToHost);
    if (e == hipSuccess) {
        const double lanes = double(grid) * 256.0;
        const double steps = double(iters) * kUnroll;
        double ops;
        if (kind == 5)  // 4 MFMAs per step per wave, 32 x 32 x 32 MACs each
            ops = double(grid) * 4.0 * steps * 4.0 * 32.0 * 32.0 * 32.0;
        else
            ops = lanes * steps * kChains;
        *seconds = ms * 1e-3;
        *ops_per_s = ops / (*seconds);
        *clock_hz = c[1] ? double(c[0]) / (double(c[1]) * 1e-8) : 0.0;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(out);
    (void)hipFree(clk);
    return int(e);
}
