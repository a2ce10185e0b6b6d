// Backward and gW-reduction launchers for storage type double.
#include "gtt_bwd.hpp"

GTT_BWD_INSTANTIATE(f64, double)
