// Ragged-batch launchers for storage type f16.
#include "gtt_inst.hpp"

GTT_RAGGED_INSTANTIATE(f16, f16)
