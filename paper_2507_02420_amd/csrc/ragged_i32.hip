// Ragged-batch launchers for storage type int32_t.
#include "gtt_inst.hpp"

GTT_RAGGED_INSTANTIATE(i32, int32_t)
