// Dominant-coefficient selection and sparse scatter, every storage type.
#include "gtt_launch.hpp"
#include "gtt_topk.hpp"

namespace gtt {

template <typename T>
static hipError_t topk_t(const void* coef, int64_t N, int64_t batch, int64_t k, int64_t* idx, void* val,
                         void* recon, hipStream_t s) {
    hipLaunchKernelGGL(gtt_topk_kernel<T>, dim3((unsigned)batch), dim3(kTopkThreads), 0, s,
                       static_cast<const T*>(coef), N, k, idx, static_cast<T*>(val));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !recon) return e;
    const int64_t E = N * batch;
    const unsigned gz = (unsigned)std::min<int64_t>((E + 255) / 256, 65536);
    hipLaunchKernelGGL(gtt_zero_kernel<T>, dim3(gz), dim3(256), 0, s, static_cast<T*>(recon), E);
    const unsigned gs = (unsigned)std::min<int64_t>((batch * k + 255) / 256, 65536);
    hipLaunchKernelGGL(gtt_scatter_kernel<T>, dim3(gs), dim3(256), 0, s, static_cast<T*>(recon), N, k, batch, idx,
                       static_cast<const T*>(val));
    return hipGetLastError();
}

hipError_t launch_topk(DT dt, const void* coef, int64_t N, int64_t batch, int64_t k, int64_t* idx, void* val,
                       void* recon, hipStream_t s) {
    switch (dt) {
        case DT::F64: return topk_t<double>(coef, N, batch, k, idx, val, recon, s);
        case DT::F32: return topk_t<float>(coef, N, batch, k, idx, val, recon, s);
        case DT::C128: return topk_t<cd>(coef, N, batch, k, idx, val, recon, s);
        case DT::C64: return topk_t<cf>(coef, N, batch, k, idx, val, recon, s);
        case DT::BF16: return topk_t<bf16>(coef, N, batch, k, idx, val, recon, s);
        case DT::F16: return topk_t<f16>(coef, N, batch, k, idx, val, recon, s);
        case DT::I32: return topk_t<int32_t>(coef, N, batch, k, idx, val, recon, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace gtt
