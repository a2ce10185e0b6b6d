// Backward and gW-reduction launchers for storage type bf16.
#include "gtt_bwd.hpp"

GTT_BWD_INSTANTIATE(bf16, bf16)
