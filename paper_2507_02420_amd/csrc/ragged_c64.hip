// Ragged-batch kernel for storage type cf.
#include "gtt_launch.hpp"
#include "gtt_ragged.hpp"

namespace gtt {

hipError_t launch_ragged_c64(const RaggedArgs& a, unsigned grid, size_t lds, hipStream_t s) {
    const void* k = reinterpret_cast<const void*>(gtt_ragged_kernel<cf>);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(gtt_ragged_kernel<cf>, dim3(grid), dim3(kThreads), lds, s, a);
    return hipGetLastError();
}

hipError_t ragged_occupancy_c64(size_t lds, int* blocks_per_cu) {
    const void* k = reinterpret_cast<const void*>(gtt_ragged_kernel<cf>);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, gtt_ragged_kernel<cf>, kThreads, lds);
}

}  // namespace gtt
