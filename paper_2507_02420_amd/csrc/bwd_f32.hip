// Instantiations of the backward and reduction kernels for storage type float.
#include "gtt_bwd.hpp"
#include "gtt_launch.hpp"

namespace gtt {

hipError_t launch_bwd_f32(const BwdArgs& a, unsigned grid, size_t lds, hipStream_t s) {
    using T = float;
    const void* k = a.b <= 8 ? reinterpret_cast<const void*>(gtt_bwd_kernel<T, 8>)
                             : reinterpret_cast<const void*>(gtt_bwd_kernel<T, 16>);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    if (a.b <= 8)
        hipLaunchKernelGGL((gtt_bwd_kernel<T, 8>), dim3(grid), dim3(kThreads), lds, s, a);
    else
        hipLaunchKernelGGL((gtt_bwd_kernel<T, 16>), dim3(grid), dim3(kThreads), lds, s, a);
    return hipGetLastError();
}

static constexpr int kReduceBlocks = 64;

hipError_t launch_reduce_f32(const void* partials, int64_t nparts, int bb, void* out, hipStream_t s) {
    using C = typename Tr<float>::C;
    // partials has room for kReduceBlocks more vectors after the nparts ones
    C* mid = const_cast<C*>(static_cast<const C*>(partials)) + (size_t)nparts * bb;
    const int g1 = (int)(nparts < kReduceBlocks ? nparts : kReduceBlocks);
    hipLaunchKernelGGL(gtt_reduce_kernel<C>, dim3(g1), dim3(kThreads), 0, s, static_cast<const C*>(partials),
                       nparts, bb, mid);
    hipLaunchKernelGGL(gtt_reduce_kernel<C>, dim3(1), dim3(kThreads), 0, s, mid, (int64_t)g1, bb,
                       static_cast<C*>(out));
    return hipGetLastError();
}

}  // namespace gtt
