// hipemu.hpp -- what the CPU emulation of the HIP runtime tells its test driver
// (test infrastructure only; see hipemu.cpp).
#pragma once

#include <stdint.h>

#include "zmc.h"

namespace hipemu {

// The result the emulated batched path gives for f evaluated in FP32 (fp64 =
// false) or FP64: sums of the emulated per-segment values, finalized by the
// library's formulas (mean V S1 / N, SE from the unbiased variance).
mc_result expected_batched(const mc_function& f, bool fp64);

// The same for the emulated plain one-launch-per-function path.
mc_result expected_plain(const mc_function& f);

// Kernels the emulation has run so far (direct launches and graph replays).
uint64_t kernel_launches();

// Calls into the emulated HIP runtime so far (an upper bound on the library's
// checked HIP calls over the same span).
uint64_t api_calls();

}  // namespace hipemu
