// Digit-group pass launchers for storage type double.
#include "gtt_inst.hpp"

GTT_PASS_INSTANTIATE(f64, double)
