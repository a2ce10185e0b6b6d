// Ragged-batch kernel for storage type bf16.
#include "gtt_launch.hpp"
#include "gtt_ragged.hpp"

namespace gtt {

hipError_t launch_ragged_bf16(const RaggedArgs& a, unsigned grid, size_t lds, hipStream_t s) {
    const void* k = reinterpret_cast<const void*>(gtt_ragged_kernel<bf16>);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(gtt_ragged_kernel<bf16>, dim3(grid), dim3(kThreads), lds, s, a);
    return hipGetLastError();
}

hipError_t ragged_occupancy_bf16(size_t lds, int* blocks_per_cu) {
    const void* k = reinterpret_cast<const void*>(gtt_ragged_kernel<bf16>);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, gtt_ragged_kernel<bf16>, kThreads, lds);
}

// one item class per launch (see ragged_class)
hipError_t launch_ragged_cls_bf16(int cls, const RaggedArgs& a, unsigned grid, size_t lds, hipStream_t s) {
    hipError_t e = hipSuccess;
#define K_(CLS)                                                                                           \
    do {                                                                                                  \
        const void* k = reinterpret_cast<const void*>(gtt_ragged_class_kernel<bf16, CLS>);                  \
        if (lds > 65536) e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
        if (e != hipSuccess) return e;                                                                    \
        /* matrix-core classes loop over their items on a resident grid */                        \
        const unsigned g = CLS >= 16 ? resident_grid((gtt_ragged_class_kernel<bf16, CLS>), kThreads, lds, grid) : grid; \
        hipLaunchKernelGGL((gtt_ragged_class_kernel<bf16, CLS>), dim3(g), dim3(kThreads), lds, s, a);    \
    } while (0)
    switch (cls) {
        case 0: K_(0); break;
        case 2: K_(2); break;
        case 3: K_(3); break;
        case 4: K_(4); break;
        case 5: K_(5); break;
        case 16: K_(16); break;
        case 32: K_(32); break;
        default: return hipErrorInvalidValue;
    }
#undef K_
    return hipGetLastError();
}

}  // namespace gtt
