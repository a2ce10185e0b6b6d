// Instantiations of the digit-group pass kernels for storage type float.
#include "gtt_launch.hpp"
#include "gtt_mfma.hpp"
#include "gtt_pass.hpp"

namespace gtt {

template <typename K>
static hipError_t set_lds(K kernel, size_t lds) {
    if (lds > 65536) return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    return hipSuccess;
}

hipError_t launch_pass_f32(int b, int kind, const PassArgs& a, unsigned grid, size_t lds, hipStream_t s) {
    using T = float;
    hipError_t e = hipSuccess;
#define GTT_LAUNCH(KER)                                                       \
    do {                                                                      \
        e = set_lds(KER, lds);                                                \
        if (e != hipSuccess) return e;                                        \
        hipLaunchKernelGGL(KER, dim3(grid), dim3(kThreads), lds, s, a);       \
    } while (0)
    // the VALU pass kernels that prefetch run a persistent grid
#define GTT_LAUNCH_VALU(B)                                                                    \
    do {                                                                                      \
        e = set_lds((gtt_pass_kernel<T, B>), lds);                                            \
        if (e != hipSuccess) return e;                                                        \
        const unsigned g = pass_prefetches<typename Tr<T>::C, B>()                            \
                               ? resident_grid((gtt_pass_kernel<T, B>), kThreads, lds, grid)  \
                               : grid;                                                        \
        hipLaunchKernelGGL((gtt_pass_kernel<T, B>), dim3(g), dim3(kThreads), lds, s, a);      \
    } while (0)
#define GTT_LAUNCH_MFMA(B)                                                                        \
    do {                                                                                          \
        e = set_lds((gtt_pass_mfma_kernel<T, B>), lds);                                           \
        if (e != hipSuccess) return e;                                                            \
        const unsigned g = resident_grid((gtt_pass_mfma_kernel<T, B>), kThreads, lds, grid);     \
        hipLaunchKernelGGL((gtt_pass_mfma_kernel<T, B>), dim3(g), dim3(kThreads), lds, s, a);     \
    } while (0)
    if (kind == kKindGeneric) {
        GTT_LAUNCH(gtt_pass_generic_kernel<T>);
    } else if (kind == kKindMfma) {
        // persistent grid: the kernel prefetches the next tile
        if (b == 16)
            GTT_LAUNCH_MFMA(16);
        else if (b == 32)
            GTT_LAUNCH_MFMA(32);
        else
            return hipErrorInvalidValue;
    } else {
        switch (b) {
            case 2: GTT_LAUNCH_VALU(2); break;
            case 3: GTT_LAUNCH_VALU(3); break;
            case 4: GTT_LAUNCH_VALU(4); break;
            case 5: GTT_LAUNCH_VALU(5); break;
            case 6: GTT_LAUNCH_VALU(6); break;
            case 7: GTT_LAUNCH_VALU(7); break;
            case 8: GTT_LAUNCH_VALU(8); break;
            default: GTT_LAUNCH(gtt_pass_generic_kernel<T>); break;
        }
    }
#undef GTT_LAUNCH
#undef GTT_LAUNCH_VALU
#undef GTT_LAUNCH_MFMA
    return hipGetLastError();
}

}  // namespace gtt
