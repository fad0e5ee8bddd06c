// The fixed device scratch used by dfr_reproject_noalloc (scratch.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace dfr {

// Size of the per-device scratch array: the cell-model table of the FP32
// forward (112 B per 32x32 output cell) fits up to 74,898 cells, e.g. an
// 8192 x 8192 output (65,536 cells).
constexpr size_t kScratchBytes = size_t(8) << 20;

// Device address of the current device's scratch array (looked up on the
// first call per device, with that device current, then cached).
hipError_t scratch_address(void **ptr);

}  // namespace dfr
