// Storage conversions between the 16-bit storage types and float32 (round to
// nearest even towards the 16-bit type), for plans that keep the values
// between digit groups in float32.
#include "gtt_launch.hpp"
#include "gtt_types.hpp"

namespace gtt {

template <typename S, typename D>
__global__ __launch_bounds__(256) void gtt_convert_kernel(const S* __restrict__ in, D* __restrict__ out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        out[i] = from_c<D>(to_c(in[i]));
}

template <typename S, typename D>
static hipError_t convert_t(const void* in, void* out, int64_t n, hipStream_t s) {
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 1 << 16));
    hipLaunchKernelGGL((gtt_convert_kernel<S, D>), dim3(grid), dim3(256), 0, s, static_cast<const S*>(in),
                       static_cast<D*>(out), n);
    return hipGetLastError();
}

hipError_t launch_convert(DT from, DT to, const void* in, void* out, int64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (from == DT::BF16 && to == DT::F32) return convert_t<bf16, float>(in, out, n, s);
    if (from == DT::F16 && to == DT::F32) return convert_t<f16, float>(in, out, n, s);
    if (from == DT::F32 && to == DT::BF16) return convert_t<float, bf16>(in, out, n, s);
    if (from == DT::F32 && to == DT::F16) return convert_t<float, f16>(in, out, n, s);
    return hipErrorInvalidValue;
}

}  // namespace gtt
