// Digit-group pass launchers for storage type int32_t.
#include "gtt_inst.hpp"

GTT_PASS_INSTANTIATE(i32, int32_t)
