// Backward and gW-reduction launchers for storage type cf.
#include "gtt_bwd.hpp"

GTT_BWD_INSTANTIATE(c64, cf)
