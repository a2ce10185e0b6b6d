// Ragged-batch launchers for storage type double.
#include "gtt_inst.hpp"

GTT_RAGGED_INSTANTIATE(f64, double)
