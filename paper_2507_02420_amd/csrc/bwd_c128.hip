// Backward and gW-reduction launchers for storage type cd.
#include "gtt_bwd.hpp"

GTT_BWD_INSTANTIATE(c128, cd)
