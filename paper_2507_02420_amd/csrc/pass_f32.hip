// Digit-group pass launchers for storage type float.
#include "gtt_inst.hpp"

GTT_PASS_INSTANTIATE(f32, float)
