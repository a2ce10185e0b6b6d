// Launchers of the complex64 radix-8 matrix-core kernels (forward /
// adjoint passes and backward, general and per-lane-address forms).
#include "gtt_launch.hpp"
#include "gtt_cmfma.hpp"

namespace gtt {

template <typename K>
static hipError_t set_lds(K kernel, size_t lds) {
    if (lds > 65536) return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    return hipSuccess;
}

// general radix-8 pass (tiles without a per-lane layout)
hipError_t launch_cpass8(const PassArgs& a, unsigned grid, size_t lds, hipStream_t s) {
    hipError_t e = set_lds(gtt_c64_mfma8_pass_kernel, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gtt_c64_mfma8_pass_kernel, dim3(grid), dim3(kThreads), lds, s, a);
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

// LDS layouts that the planner produces for the complex radix-8 groups of
// the 256 x 8^6 workload (four digits of 4096-element contiguous tiles, two
// digits of 64-column strided tiles), compiled with fixed offsets; every
// other layout runs the same kernels with run-time offsets.  A host test
// checks that the planner still produces exactly these layouts.
using FwdLay4 = LayoutFixed<0x1f0a05, 0, 0x1e001b00270017ull>;
using FwdLay2 = LayoutFixed<0x1f0a05, 6, 0x1e001bull>;
using BwdLay4 = LayoutFixed<0x1f0805, 0, 0x81b031b01870887ull, 0x7878u>;
using BwdLay2 = LayoutFixed<0x1f0905, 6, 0x31d081bull>;

template <class LAY>
static bool layout_is(const PassArgs& a) {
    return a.pad_shift == LAY::kPad && a.logC == LAY::kLogC && a.fmap == LAY::kFmap && a.pmap == LAY::kPmap;
}

template <int K, int NI, class LAY>
static hipError_t launch_pfast(const PassArgs& a, unsigned grid, size_t lds, hipStream_t s) {
    hipError_t e = set_lds(gtt_c64_mfma8_pass_fast_kernel<K, NI, LAY>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((gtt_c64_mfma8_pass_fast_kernel<K, NI, LAY>), dim3(grid), dim3(kBwdThreads), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_cpass8_fast(int k, int ni, const PassArgs& a, unsigned grid, size_t lds, hipStream_t s) {
    if (k == 4 && ni == 2 && layout_is<FwdLay4>(a)) return launch_pfast<4, 2, FwdLay4>(a, grid, lds, s);
    if (k == 2 && ni == 2 && layout_is<FwdLay2>(a)) return launch_pfast<2, 2, FwdLay2>(a, grid, lds, s);
    switch (k * 4 + ni) {
        case 1 * 4 + 1: return launch_pfast<1, 1, LayoutArgs>(a, grid, lds, s);
        case 1 * 4 + 2: return launch_pfast<1, 2, LayoutArgs>(a, grid, lds, s);
        case 2 * 4 + 1: return launch_pfast<2, 1, LayoutArgs>(a, grid, lds, s);
        case 2 * 4 + 2: return launch_pfast<2, 2, LayoutArgs>(a, grid, lds, s);
        case 3 * 4 + 1: return launch_pfast<3, 1, LayoutArgs>(a, grid, lds, s);
        case 3 * 4 + 2: return launch_pfast<3, 2, LayoutArgs>(a, grid, lds, s);
        case 4 * 4 + 1: return launch_pfast<4, 1, LayoutArgs>(a, grid, lds, s);
        case 4 * 4 + 2: return launch_pfast<4, 2, LayoutArgs>(a, grid, lds, s);
        default: return hipErrorInvalidValue;
    }
}

template <int K, int NI, class LAY, bool D0 = false>
static hipError_t launch_fast(const CBwdArgs& a, unsigned grid, size_t lds, hipStream_t s) {
    hipError_t e = set_lds(gtt_c64_mfma8_bwd_fast_kernel<K, NI, LAY, D0>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((gtt_c64_mfma8_bwd_fast_kernel<K, NI, LAY, D0>), dim3(grid), dim3(kBwdThreads), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_cbwd8_fast(int k, int ni, const CBwdArgs& a, unsigned grid, size_t lds, hipStream_t s) {
    // contiguous tiles with digit 0 at stride 1: input and gx move in the
    // digit-0 pass layout
    if (k == 4 && ni == 2 && layout_is<BwdLay4>(a.p) && a.p.mode == kContigVec)
        return launch_fast<4, 2, BwdLay4, true>(a, grid, lds, s);
    if (k == 4 && ni == 2 && layout_is<BwdLay4>(a.p)) return launch_fast<4, 2, BwdLay4>(a, grid, lds, s);
    if (k == 2 && ni == 2 && layout_is<BwdLay2>(a.p)) return launch_fast<2, 2, BwdLay2>(a, grid, lds, s);
    switch (k * 4 + ni) {
        case 1 * 4 + 1: return launch_fast<1, 1, LayoutArgs>(a, grid, lds, s);
        case 1 * 4 + 2: return launch_fast<1, 2, LayoutArgs>(a, grid, lds, s);
        case 2 * 4 + 1: return launch_fast<2, 1, LayoutArgs>(a, grid, lds, s);
        case 2 * 4 + 2: return launch_fast<2, 2, LayoutArgs>(a, grid, lds, s);
        case 3 * 4 + 1: return launch_fast<3, 1, LayoutArgs>(a, grid, lds, s);
        case 3 * 4 + 2: return launch_fast<3, 2, LayoutArgs>(a, grid, lds, s);
        case 4 * 4 + 1: return launch_fast<4, 1, LayoutArgs>(a, grid, lds, s);
        case 4 * 4 + 2: return launch_fast<4, 2, LayoutArgs>(a, grid, lds, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace gtt
