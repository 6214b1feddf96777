// qedx_scratch.hpp -- fixed per-device scratch of the allocation-free entry
// point (defined in qedx_scratch.hip, the library's one HIP-compiled unit).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace qedx_rt {
// Size of the scratch array each device holds.
constexpr int64_t kScratchBytes = (int64_t)256 << 20;
// Device address of the current device's scratch array, resolved with
// hipGetSymbolAddress on the first call per device and cached.
hipError_t scratch_address(void** out);
}  // namespace qedx_rt
