// Ragged-batch launchers for storage type cd.
#include "gtt_inst.hpp"

GTT_RAGGED_INSTANTIATE(c128, cd)
