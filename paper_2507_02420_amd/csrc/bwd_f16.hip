// Backward and gW-reduction launchers for storage type f16.
#include "gtt_bwd.hpp"

GTT_BWD_INSTANTIATE(f16, f16)
