// Host launchers of the digit-group pass and ragged-batch kernels, written
// once as templates over the storage type; each pass_<dtype>.hip and
// ragged_<dtype>.hip translation unit instantiates them for one storage type
// (GTT_PASS_INSTANTIATE / GTT_RAGGED_INSTANTIATE), so the dtypes compile in
// parallel.
#pragma once

#include <type_traits>

#include "gtt_launch.hpp"
#include "gtt_mfma.hpp"
#include "gtt_pass.hpp"
#include "gtt_ragged.hpp"

namespace gtt {

// matrix-core pass kernels exist for 16-bit and float storage
template <typename T>
constexpr bool has_mfma_pass() {
    return sizeof(T) == 2 || std::is_same<T, float>::value;
}
// the VALU pass kernels hold W in registers: radix <= 8, complex double <= 5
template <typename T>
constexpr int valu_max_radix() {
    return std::is_same<T, cd>::value ? 5 : 8;
}

template <typename K>
inline hipError_t set_lds(K kernel, size_t lds) {
    if (lds > 65536)
        return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds);
    return hipSuccess;
}

// one tile per work-group
template <typename K>
inline hipError_t launch_tiles(K kernel, const PassArgs& a, unsigned grid, size_t lds, hipStream_t s) {
    hipError_t e = set_lds(kernel, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(kThreads), lds, s, a);
    return hipGetLastError();
}

// VALU pass of radix B: the kernels that prefetch the next tile run a
// persistent grid (occupancy x compute units)
template <typename T, int B>
inline hipError_t launch_valu(const PassArgs& a, unsigned grid, size_t lds, hipStream_t s) {
    hipError_t e = set_lds(gtt_pass_kernel<T, B>, lds);
    if (e != hipSuccess) return e;
    const unsigned g =
        pass_prefetches<typename Tr<T>::C, B>() ? resident_grid(gtt_pass_kernel<T, B>, kThreads, lds, grid) : grid;
    hipLaunchKernelGGL((gtt_pass_kernel<T, B>), dim3(g), dim3(kThreads), lds, s, a);
    return hipGetLastError();
}

// matrix-core pass of radix B: a persistent grid, the kernel prefetches the
// next tile
template <typename T, int B>
inline hipError_t launch_mfma(const PassArgs& a, unsigned grid, size_t lds, hipStream_t s) {
    hipError_t e = set_lds(gtt_pass_mfma_kernel<T, B>, lds);
    if (e != hipSuccess) return e;
    const unsigned g = resident_grid(gtt_pass_mfma_kernel<T, B>, kThreads, lds, grid);
    hipLaunchKernelGGL((gtt_pass_mfma_kernel<T, B>), dim3(g), dim3(kThreads), lds, s, a);
    return hipGetLastError();
}

// runtime-radix pass: the form with the scalar address walk for element-wise
// tiles
template <typename T>
inline hipError_t launch_generic(const PassArgs& a, unsigned grid, size_t lds, hipStream_t s) {
    if (a.mode == kContigScalar || a.mode == kRowScalar)
        return launch_tiles(gtt_pass_generic_kernel<T, true>, a, grid, lds, s);
    return launch_tiles(gtt_pass_generic_kernel<T, false>, a, grid, lds, s);
}

template <typename T>
hipError_t launch_pass_t(int b, int kind, const PassArgs& a, unsigned grid, size_t lds, hipStream_t s) {
    if (kind == kKindGeneric) return launch_generic<T>(a, grid, lds, s);
    if (kind == kKindMfma) {
        if constexpr (has_mfma_pass<T>()) {
            if (b == 16) return launch_mfma<T, 16>(a, grid, lds, s);
            if (b == 32) return launch_mfma<T, 32>(a, grid, lds, s);
        }
        return hipErrorInvalidValue;
    }
    if (kind == kKindCMfma) {
        if constexpr (std::is_same<T, cf>::value) {
            if (b == 8) return launch_cpass8(a, grid, lds, s);
        }
        return hipErrorInvalidValue;
    }
    constexpr int mx = valu_max_radix<T>();
    switch (b) {
        case 2:
            if (wave2_ok<T>(a)) {
                // one wave per 1024 elements, four waves a work-group
                const int64_t E = a.ntiles * (int64_t)a.P * (int64_t)a.G;
                const int64_t wg = ((E + 1023) / 1024 + kThreads / 64 - 1) / (kThreads / 64);
                const unsigned g = (unsigned)std::min<int64_t>(std::max<int64_t>(wg, 1), 1 << 20);
                hipLaunchKernelGGL(gtt_pass_wave2_kernel<T>, dim3(g), dim3(kThreads), 0, s, a);
                return hipGetLastError();
            }
            return launch_valu<T, 2>(a, grid, lds, s);
        case 3: return launch_valu<T, 3>(a, grid, lds, s);
        case 4: return launch_valu<T, 4>(a, grid, lds, s);
        case 5: return launch_valu<T, 5>(a, grid, lds, s);
        case 6: if constexpr (mx >= 6) return launch_valu<T, mx >= 6 ? 6 : 2>(a, grid, lds, s); break;
        case 7: if constexpr (mx >= 7) return launch_valu<T, mx >= 7 ? 7 : 2>(a, grid, lds, s); break;
        case 8: if constexpr (mx >= 8) return launch_valu<T, mx >= 8 ? 8 : 2>(a, grid, lds, s); break;
        default: break;
    }
    return launch_generic<T>(a, grid, lds, s);
}

// ---- ragged batches --------------------------------------------------------
template <typename T>
hipError_t launch_ragged_t(const RaggedArgs& a, unsigned grid, size_t lds, hipStream_t s) {
    hipError_t e = set_lds(gtt_ragged_kernel<T>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gtt_ragged_kernel<T>, dim3(grid), dim3(kThreads), lds, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t ragged_occupancy_t(size_t lds, int* blocks_per_cu) {
    hipError_t e = set_lds(gtt_ragged_kernel<T>, lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, gtt_ragged_kernel<T>, kThreads, lds);
}

// one item class per launch (see ragged_class); matrix-core classes loop
// over their items on a resident grid
template <typename T, int CLS>
inline hipError_t launch_ragged_class(const RaggedArgs& a, unsigned grid, size_t lds, hipStream_t s) {
    hipError_t e = set_lds(gtt_ragged_class_kernel<T, CLS>, lds);
    if (e != hipSuccess) return e;
    const unsigned g = CLS >= 16 ? resident_grid(gtt_ragged_class_kernel<T, CLS>, kThreads, lds, grid) : grid;
    hipLaunchKernelGGL((gtt_ragged_class_kernel<T, CLS>), dim3(g), dim3(kThreads), lds, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ragged_cls_t(int cls, const RaggedArgs& a, unsigned grid, size_t lds, hipStream_t s) {
    switch (cls) {
        case 0: return launch_ragged_class<T, 0>(a, grid, lds, s);
        case 2: return launch_ragged_class<T, 2>(a, grid, lds, s);
        case 3: return launch_ragged_class<T, 3>(a, grid, lds, s);
        case 4: return launch_ragged_class<T, 4>(a, grid, lds, s);
        case 5: return launch_ragged_class<T, 5>(a, grid, lds, s);
        case 16:
            if constexpr (has_mfma_pass<T>()) return launch_ragged_class<T, has_mfma_pass<T>() ? 16 : 0>(a, grid, lds, s);
            break;
        case 32:
            if constexpr (has_mfma_pass<T>()) return launch_ragged_class<T, has_mfma_pass<T>() ? 32 : 0>(a, grid, lds, s);
            break;
        default: break;
    }
    return hipErrorInvalidValue;
}

}  // namespace gtt

#define GTT_PASS_INSTANTIATE(NAME, T)                                                                   \
    namespace gtt {                                                                                     \
    hipError_t launch_pass_##NAME(int b, int kind, const PassArgs& a, unsigned grid, size_t lds,        \
                                  hipStream_t s) {                                                      \
        return launch_pass_t<T>(b, kind, a, grid, lds, s);                                              \
    }                                                                                                   \
    }

#define GTT_RAGGED_INSTANTIATE(NAME, T)                                                                 \
    namespace gtt {                                                                                     \
    hipError_t launch_ragged_##NAME(const RaggedArgs& a, unsigned grid, size_t lds, hipStream_t s) {    \
        return launch_ragged_t<T>(a, grid, lds, s);                                                     \
    }                                                                                                   \
    hipError_t ragged_occupancy_##NAME(size_t lds, int* blocks_per_cu) {                                \
        return ragged_occupancy_t<T>(lds, blocks_per_cu);                                               \
    }                                                                                                   \
    hipError_t launch_ragged_cls_##NAME(int cls, const RaggedArgs& a, unsigned grid, size_t lds,        \
                                        hipStream_t s) {                                                \
        return launch_ragged_cls_t<T>(cls, a, grid, lds, s);                                            \
    }                                                                                                   \
    }
