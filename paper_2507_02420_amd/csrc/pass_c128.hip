// Digit-group pass launchers for storage type cd.
#include "gtt_inst.hpp"

GTT_PASS_INSTANTIATE(c128, cd)
