// Ragged-batch launchers for storage type cf.
#include "gtt_inst.hpp"

GTT_RAGGED_INSTANTIATE(c64, cf)
