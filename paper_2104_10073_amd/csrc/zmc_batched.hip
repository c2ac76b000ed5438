// zmc_batched.hip -- the persistent batched kernels for the four built-in
// families, FP32 and FP64 evaluation (the hot path: Philox samples, box mapping,
// integrand, compensated sums, segment and tile reductions).  The device code is
// in zmc_device_code.hpp; this file only instantiates it.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "zmc_device_code.hpp"

namespace zmc {

extern "C" __global__ __launch_bounds__(kBlockThreads) void zmc_batched_fp32(const LaunchDesc* __restrict__ Ld)
{
    batched_body<BuiltinDispatch<false>>(Ld, kKernelBuiltin32);
}

extern "C" __global__ __launch_bounds__(kBlockThreads) void zmc_batched_fp64(const LaunchDesc* __restrict__ Ld)
{
    batched_body<BuiltinDispatch<true>>(Ld, kKernelBuiltin64);
}

// The resident kernel (the resident engine's protocol and loop are in
// zmc_device_code.hpp, shared with the resident kernels compiled at run time
// for contexts with caller families).
extern "C" __global__ __launch_bounds__(kBlockThreads) void zmc_resident(const ResidentDesc* __restrict__ R, uint32_t epoch)
{
    resident_body<BuiltinDispatch<false>, BuiltinDispatch<true>>(R, epoch);
}

const void* batched_kernel_ptr(bool fp64) { return fp64 ? (const void*)zmc_batched_fp64 : (const void*)zmc_batched_fp32; }
const void* resident_kernel_ptr() { return (const void*)zmc_resident; }

}  // namespace zmc
