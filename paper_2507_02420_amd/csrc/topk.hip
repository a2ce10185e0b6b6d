// Dominant-coefficient selection and sparse scatter, every storage type.
#include "gtt_launch.hpp"
#include "gtt_topk.hpp"

namespace gtt {

template <typename T>
static hipError_t topk_chunked_t(const T* coef, int64_t N, int64_t batch, int64_t k, int64_t* idx, T* val,
                                 T* recon, void* meta, hipStream_t s) {
    using K = typename TopkKey<T>::K;
    const int64_t nch = (N + kTopkChunk - 1) / kTopkChunk;
    auto r = [](size_t x) { return (x + 255) & ~(size_t)255; };
    char* m = static_cast<char*>(meta);
    TopkState* st = reinterpret_cast<TopkState*>(m);
    m += r((size_t)batch * sizeof(TopkState));
    uint32_t* ghist = reinterpret_cast<uint32_t*>(m);
    m += r((size_t)batch * 256 * 4);
    uint32_t* cnt = reinterpret_cast<uint32_t*>(m);
    m += r((size_t)(batch * nch) * 8);
    int64_t* off = reinterpret_cast<int64_t*>(m);
    const dim3 grid((unsigned)nch, (unsigned)batch);
    hipLaunchKernelGGL(gtt_topk_init_kernel<K>, dim3((unsigned)batch), dim3(256), 0, s, st, ghist, batch, k);
    for (int shift = 8 * (int)sizeof(K) - 8; shift >= 0; shift -= 8) {
        hipLaunchKernelGGL(gtt_topk_hist_kernel<T>, grid, dim3(kTopkChunkThreads), 0, s, coef, N,
                           (const TopkState*)st, ghist, shift);
        hipLaunchKernelGGL(gtt_topk_select_kernel<K>, dim3((unsigned)batch), dim3(256), 0, s, st, ghist, shift);
    }
    hipLaunchKernelGGL(gtt_topk_count_kernel<T>, grid, dim3(kTopkChunkThreads), 0, s, coef, N, nch,
                       (const TopkState*)st, cnt);
    hipLaunchKernelGGL(gtt_topk_scan_kernel, dim3((unsigned)batch), dim3(256), 0, s, (const TopkState*)st,
                       (const uint32_t*)cnt, off, nch);
    hipLaunchKernelGGL(gtt_topk_write_kernel<T>, grid, dim3(kTopkChunkThreads), 0, s, coef, N, nch,
                       (const TopkState*)st, (const int64_t*)off, k, idx, val, recon);
    return hipGetLastError();
}

template <typename T>
static hipError_t topk_t(const void* coef, int64_t N, int64_t batch, int64_t k, int64_t* idx, void* val,
                         void* recon, void* meta, hipStream_t s) {
    hipError_t e;
    if (topk_chunked(N, batch)) {
        // the ordered write also fills the dense sparse vector
        return topk_chunked_t<T>(static_cast<const T*>(coef), N, batch, k, idx, static_cast<T*>(val),
                                 static_cast<T*>(recon), meta, s);
    } else {
        hipLaunchKernelGGL(gtt_topk_kernel<T>, dim3((unsigned)batch), dim3(kTopkThreads), 0, s,
                           static_cast<const T*>(coef), N, k, idx, static_cast<T*>(val));
        e = hipGetLastError();
    }
    if (e != hipSuccess || !recon) return e;
    const int64_t E = N * batch;
    const unsigned gz = (unsigned)std::min<int64_t>((E + 255) / 256, 65536);
    hipLaunchKernelGGL(gtt_zero_kernel<T>, dim3(gz), dim3(256), 0, s, static_cast<T*>(recon), E);
    const unsigned gs = (unsigned)std::min<int64_t>((batch * k + 255) / 256, 65536);
    hipLaunchKernelGGL(gtt_scatter_kernel<T>, dim3(gs), dim3(256), 0, s, static_cast<T*>(recon), N, k, batch, idx,
                       static_cast<const T*>(val));
    return hipGetLastError();
}

size_t topk_meta_bytes(int64_t N, int64_t batch) { return topk_ws_bytes(N, batch); }

hipError_t launch_topk(DT dt, const void* coef, int64_t N, int64_t batch, int64_t k, int64_t* idx, void* val,
                       void* recon, void* meta, hipStream_t s) {
    switch (dt) {
        case DT::F64: return topk_t<double>(coef, N, batch, k, idx, val, recon, meta, s);
        case DT::F32: return topk_t<float>(coef, N, batch, k, idx, val, recon, meta, s);
        case DT::C128: return topk_t<cd>(coef, N, batch, k, idx, val, recon, meta, s);
        case DT::C64: return topk_t<cf>(coef, N, batch, k, idx, val, recon, meta, s);
        case DT::BF16: return topk_t<bf16>(coef, N, batch, k, idx, val, recon, meta, s);
        case DT::F16: return topk_t<f16>(coef, N, batch, k, idx, val, recon, meta, s);
        case DT::I32: return topk_t<int32_t>(coef, N, batch, k, idx, val, recon, meta, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace gtt
