// Digit-group pass launchers for storage type f16.
#include "gtt_inst.hpp"

GTT_PASS_INSTANTIATE(f16, f16)
