// Host-side launch entry points of the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>

#include "gtt_args.hpp"

namespace gtt {

enum class DT : int { F64 = 0, F32 = 1, C128 = 2, C64 = 3, BF16 = 4, F16 = 5, I32 = 6 };

// forward / inverse digit-group pass (specialised radix 2..8, else the
// runtime-radix kernel; `generic` forces the runtime-radix kernel)
hipError_t launch_pass(DT dt, int b, bool generic, const PassArgs& a, unsigned grid, size_t lds,
                       hipStream_t s);

}  // namespace gtt
