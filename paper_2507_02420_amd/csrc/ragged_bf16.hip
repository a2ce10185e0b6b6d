// Ragged-batch launchers for storage type bf16.
#include "gtt_inst.hpp"

GTT_RAGGED_INSTANTIATE(bf16, bf16)
