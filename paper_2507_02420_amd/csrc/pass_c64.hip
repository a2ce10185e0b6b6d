// Digit-group pass launchers for storage type cf.
#include "gtt_inst.hpp"

GTT_PASS_INSTANTIATE(c64, cf)
