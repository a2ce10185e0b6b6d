// Instantiations of the digit-group pass kernels for storage type double.
#include "gtt_launch.hpp"
#include "gtt_pass.hpp"

namespace gtt {

template <typename K>
static hipError_t set_lds(K kernel, size_t lds) {
    if (lds > 65536) return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    return hipSuccess;
}

hipError_t launch_pass_f64(int b, int kind, const PassArgs& a, unsigned grid, size_t lds, hipStream_t s) {
    using T = double;
    hipError_t e = hipSuccess;
#define GTT_LAUNCH(KER)                                                       \
    do {                                                                      \
        e = set_lds(KER, lds);                                                \
        if (e != hipSuccess) return e;                                        \
        hipLaunchKernelGGL(KER, dim3(grid), dim3(kThreads), lds, s, a);       \
    } while (0)
    if (kind == kKindGeneric) {
        GTT_LAUNCH(gtt_pass_generic_kernel<T>);
    } else if (kind == kKindMfma) {
        return hipErrorInvalidValue;
    } else {
        switch (b) {
            case 2: GTT_LAUNCH((gtt_pass_kernel<T, 2>)); break;
            case 3: GTT_LAUNCH((gtt_pass_kernel<T, 3>)); break;
            case 4: GTT_LAUNCH((gtt_pass_kernel<T, 4>)); break;
            case 5: GTT_LAUNCH((gtt_pass_kernel<T, 5>)); break;
            case 6: GTT_LAUNCH((gtt_pass_kernel<T, 6>)); break;
            case 7: GTT_LAUNCH((gtt_pass_kernel<T, 7>)); break;
            case 8: GTT_LAUNCH((gtt_pass_kernel<T, 8>)); break;
            default: GTT_LAUNCH(gtt_pass_generic_kernel<T>); break;
        }
    }
#undef GTT_LAUNCH
    return hipGetLastError();
}

}  // namespace gtt
