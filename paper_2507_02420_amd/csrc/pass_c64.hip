// Instantiations of the digit-group pass kernels for storage type cf.
#include "gtt_launch.hpp"
#include "gtt_cmfma.hpp"
#include "gtt_pass.hpp"

namespace gtt {

template <typename K>
static hipError_t set_lds(K kernel, size_t lds) {
    if (lds > 65536) return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    return hipSuccess;
}

hipError_t launch_pass_c64(int b, int kind, const PassArgs& a, unsigned grid, size_t lds, hipStream_t s) {
    using T = cf;
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
    } else if (kind == kKindCMfma) {
        if (b != 8) return hipErrorInvalidValue;
        GTT_LAUNCH(gtt_c64_mfma8_pass_kernel<false>);
    } else {
        switch (b) {
            case 2: GTT_LAUNCH((gtt_pass_kernel<T, 2, false>)); break;
            case 3: GTT_LAUNCH((gtt_pass_kernel<T, 3, false>)); break;
            case 4: GTT_LAUNCH((gtt_pass_kernel<T, 4, false>)); break;
            case 5: GTT_LAUNCH((gtt_pass_kernel<T, 5, false>)); break;
            case 6: GTT_LAUNCH((gtt_pass_kernel<T, 6, false>)); break;
            case 7: GTT_LAUNCH((gtt_pass_kernel<T, 7, false>)); break;
            case 8: GTT_LAUNCH((gtt_pass_kernel<T, 8, false>)); break;
            default: GTT_LAUNCH(gtt_pass_generic_kernel<T>); break;
        }
    }
#undef GTT_LAUNCH
    return hipGetLastError();
}

hipError_t launch_cbwd8(const CBwdArgs& a, unsigned grid, size_t lds, hipStream_t s) {
    hipError_t e = set_lds(gtt_c64_mfma8_bwd_kernel, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gtt_c64_mfma8_bwd_kernel, dim3(grid), dim3(kBwdThreads), lds, s, a);
    return hipGetLastError();
}

template <int K, int NI>
static hipError_t launch_fast(const CBwdArgs& a, unsigned grid, size_t lds, hipStream_t s) {
    hipError_t e = set_lds(gtt_c64_mfma8_bwd_fast_kernel<K, NI>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((gtt_c64_mfma8_bwd_fast_kernel<K, NI>), dim3(grid), dim3(kBwdThreads), lds, s, a);
    return hipGetLastError();
}

template <int K, int NI>
static hipError_t launch_pfast(const PassArgs& a, unsigned grid, size_t lds, hipStream_t s) {
    hipError_t e = set_lds(gtt_c64_mfma8_pass_fast_kernel<K, NI>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((gtt_c64_mfma8_pass_fast_kernel<K, NI>), dim3(grid), dim3(kBwdThreads), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_cpass8_fast(int k, int ni, const PassArgs& a, unsigned grid, size_t lds, hipStream_t s) {
    switch (k * 4 + ni) {
        case 1 * 4 + 1: return launch_pfast<1, 1>(a, grid, lds, s);
        case 1 * 4 + 2: return launch_pfast<1, 2>(a, grid, lds, s);
        case 2 * 4 + 1: return launch_pfast<2, 1>(a, grid, lds, s);
        case 2 * 4 + 2: return launch_pfast<2, 2>(a, grid, lds, s);
        case 3 * 4 + 1: return launch_pfast<3, 1>(a, grid, lds, s);
        case 3 * 4 + 2: return launch_pfast<3, 2>(a, grid, lds, s);
        case 4 * 4 + 1: return launch_pfast<4, 1>(a, grid, lds, s);
        case 4 * 4 + 2: return launch_pfast<4, 2>(a, grid, lds, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_cbwd8_fast(int k, int ni, const CBwdArgs& a, unsigned grid, size_t lds, hipStream_t s) {
    switch (k * 4 + ni) {
        case 1 * 4 + 1: return launch_fast<1, 1>(a, grid, lds, s);
        case 1 * 4 + 2: return launch_fast<1, 2>(a, grid, lds, s);
        case 2 * 4 + 1: return launch_fast<2, 1>(a, grid, lds, s);
        case 2 * 4 + 2: return launch_fast<2, 2>(a, grid, lds, s);
        case 3 * 4 + 1: return launch_fast<3, 1>(a, grid, lds, s);
        case 3 * 4 + 2: return launch_fast<3, 2>(a, grid, lds, s);
        case 4 * 4 + 1: return launch_fast<4, 1>(a, grid, lds, s);
        case 4 * 4 + 2: return launch_fast<4, 2>(a, grid, lds, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace gtt
