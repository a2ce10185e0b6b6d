// Ragged-batch launchers for storage type float.
#include "gtt_inst.hpp"

GTT_RAGGED_INSTANTIATE(f32, float)
