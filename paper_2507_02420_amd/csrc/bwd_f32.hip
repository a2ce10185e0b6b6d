// Backward and gW-reduction launchers for storage type float.
#include "gtt_bwd.hpp"

GTT_BWD_INSTANTIATE(f32, float)
