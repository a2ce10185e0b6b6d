// Host side of backward and of the natural-order filter.
#include <hip/hip_runtime.h>

#include "gtt_launch.hpp"
#include "gtt_plan.hpp"

namespace gtt {

gtt_status backward_impl(gtt_plan_s*, const void*, const void*, const void*, const void*, void*, void*, void*,
                         size_t, hipStream_t) {
    return GTT_ERR_UNSUPPORTED;
}

gtt_status filter_impl(gtt_plan_s*, const void*, const void*, int64_t, void*, void*, void*, size_t, hipStream_t) {
    return GTT_ERR_UNSUPPORTED;
}

}  // namespace gtt
