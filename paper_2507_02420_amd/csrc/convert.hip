// Storage conversions between the 16-bit storage types and float32 (round to
// nearest even towards the 16-bit type), for plans that keep the values
// between digit groups in float32; a zero fill (gW of a transform with no
// digit) that stays a kernel node under graph capture; the reset of the
// ragged grid-barrier words.
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

__global__ __launch_bounds__(256) void gtt_zero_kernel(uint32_t* __restrict__ p, int64_t nwords) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nwords; i += (int64_t)gridDim.x * 256) p[i] = 0u;
}

// Before a persistent ragged launch: fresh arrival and generation words of
// the grid barrier; a failure of an earlier launch moves into the sticky
// record (word 3) that gtt_plan_check reads.
__global__ void gtt_barrier_reset_kernel(unsigned* bar) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (bar[2]) bar[3] = 1u;
        bar[0] = 0u;
        bar[1] = 0u;
        bar[2] = 0u;
    }
}

hipError_t launch_barrier_reset(unsigned* bar, hipStream_t s) {
    hipLaunchKernelGGL(gtt_barrier_reset_kernel, dim3(1), dim3(64), 0, s, bar);
    return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
    // every caller zeroes whole compute-dtype elements (multiples of 4 bytes)
    if (bytes == 0) return hipSuccess;
    if (bytes % 4) return hipErrorInvalidValue;
    const int64_t nw = (int64_t)(bytes / 4);
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((nw + 255) / 256, 1 << 12));
    hipLaunchKernelGGL(gtt_zero_kernel, dim3(grid), dim3(256), 0, s, static_cast<uint32_t*>(p), nw);
    return hipGetLastError();
}

}  // namespace gtt
