// Digit-group pass launchers for storage type bf16.
#include "gtt_inst.hpp"

GTT_PASS_INSTANTIATE(bf16, bf16)
