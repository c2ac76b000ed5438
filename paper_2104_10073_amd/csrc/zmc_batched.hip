// zmc_batched.hip -- the persistent batched kernels for the four built-in
// families, FP32 and FP64 evaluation (the hot path: Philox samples, box mapping,
// integrand, compensated sums, segment and tile reductions).  The device code is
// in zmc_device_code.hpp; this file only instantiates it.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "zmc_device_code.hpp"

namespace zmc {

// Family dispatch of the built-in kernels (a wave-uniform branch per tile).
template <bool F64>
struct BuiltinDispatch {
    template <int FAM>
    using Ev = typename std::conditional<F64, Eval64<FAM>, Eval32<FAM>>::type;
    __device__ static __forceinline__ bool run(CDevFn* fn, uint32_t fam, uint32_t seg0, uint32_t seg_log2,
                                               uint32_t wave, uint32_t lane, Partial* s_seg)
    {
        switch (fam) {
        case HARMONIC: tile_segments<Ev<HARMONIC>>(fn, seg0, seg_log2, wave, lane, s_seg); return true;
        case ABS_LINEAR: tile_segments<Ev<ABS_LINEAR>>(fn, seg0, seg_log2, wave, lane, s_seg); return true;
        case GAUSSIAN: tile_segments<Ev<GAUSSIAN>>(fn, seg0, seg_log2, wave, lane, s_seg); return true;
        case POLY_PRODUCT: tile_segments<Ev<POLY_PRODUCT>>(fn, seg0, seg_log2, wave, lane, s_seg); return true;
        default: return false;
        }
    }
};

extern "C" __global__ __launch_bounds__(kBlockThreads) void zmc_batched_fp32(const LaunchDesc* __restrict__ Ld)
{
    batched_body<BuiltinDispatch<false>>(Ld, kKernelBuiltin32);
}

extern "C" __global__ __launch_bounds__(kBlockThreads) void zmc_batched_fp64(const LaunchDesc* __restrict__ Ld)
{
    batched_body<BuiltinDispatch<true>>(Ld, kKernelBuiltin64);
}

const void* batched_kernel_ptr(bool fp64) { return fp64 ? (const void*)zmc_batched_fp64 : (const void*)zmc_batched_fp32; }

}  // namespace zmc
