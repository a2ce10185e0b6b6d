// Host-side launch entry points of the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <tuple>

#include "gtt_args.hpp"

namespace gtt {

enum class DT : int { F64 = 0, F32 = 1, C128 = 2, C64 = 3, BF16 = 4, F16 = 5, I32 = 6 };

// compute units of the current device (cached per device)
inline int device_cus() {
    static int cus[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    if (cus[dev] == 0) {
        int c = 0;
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess) cus[dev] = c;
    }
    return cus[dev];
}

// work-groups of a persistent launch over `tiles` tiles: as many as the
// device holds at once (occupancy x compute units), at most one per tile
// work-groups of `kernel` one compute unit holds at once (cached per kernel,
// block size and LDS size; 0 when the query fails)
inline int occupancy_cached(const void* kernel, int threads, size_t lds) {
    static std::mutex mu;
    static std::map<std::tuple<const void*, int, size_t>, int> cache;
    const auto key = std::make_tuple(kernel, threads, lds);
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, threads, lds) != hipSuccess) occ = 0;
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = occ;
    return occ;
}

template <typename K>
inline unsigned resident_grid(K kernel, int threads, size_t lds, unsigned tiles) {
    const int cus = device_cus();
    const int occ = cus > 0 ? occupancy_cached(reinterpret_cast<const void*>(kernel), threads, lds) : 0;
    if (occ < 1) return tiles;
    const unsigned long long g = (unsigned long long)occ * (unsigned long long)cus;
    return g < tiles ? (unsigned)g : tiles;
}

// kernel families of a digit-group pass
constexpr int kKindValu = 0;     // radix 2..8, register super-stages on the VALU
constexpr int kKindGeneric = 1;  // any radix <= 64 and mixed radices, LDS sweeps
constexpr int kGenericInplaceMax = 16;  // the runtime-radix kernel: radices up to this run in place
constexpr int kKindMfma = 2;     // radix 16 / 32, bf16 / f16 storage, matrix cores
constexpr int kKindCMfma = 3;    // complex64, radix 8, FP32 matrix cores

// forward / inverse digit-group pass
hipError_t launch_pass(DT dt, int b, int kind, const PassArgs& a, unsigned grid, size_t lds, hipStream_t s);

struct BwdArgs;
// backward of one digit group, floating dtypes: radix > 0 runs the
// register-block kernel of that radix (one W for every digit; the schedule
// counts blocks of bwd_block_digits digits), 0 the runtime-radix kernel
// (radices up to maxb <= 32); threads: the register-block kernel's
// work-group size, from launch_bwd_threads
hipError_t launch_bwd(DT dt, const BwdArgs& a, int maxb, int radix, unsigned grid, int threads, size_t lds,
                      hipStream_t s);
// work-group size (256, 512 or 1024) of the radix-`radix` register-block
// backward kernel with the most resident waves for `lds` bytes of LDS
// (occupancy queries on the current device, cached); kThreads for radix 0
int launch_bwd_threads(DT dt, int radix, size_t lds);
// digits per register block of the radix-b backward kernel for dtype dt (0:
// no such kernel)
int bwd_block_digits(DT dt, int b);
// gW = fixed-order sum of nparts partial vectors of bb accumulation-dtype
// values (FP64 / complex FP64), written in the compute dtype
hipError_t launch_reduce(DT dt, const void* partials, int64_t nparts, int bb, void* out, hipStream_t s);
// bytes zeros at p (a kernel, not a memset node: safe under graph capture)
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
// fresh grid-barrier words before a persistent ragged launch
hipError_t launch_barrier_reset(unsigned* bar, hipStream_t s);

struct CBwdArgs;
// backward of one digit group, complex64 radix 8 on the matrix cores
hipError_t launch_cbwd8(const CBwdArgs& a, unsigned grid, size_t lds, hipStream_t s);
// the same on tiles of 2048 * ni elements (ni = 1, 2) with k <= 4 digits,
// LDS addresses precomputed per lane
// forward / adjoint pass of k <= 4 radix-8 digits, complex64, tiles of
// 2048 * ni elements, 1024 threads, per-lane LDS addresses
hipError_t launch_cpass8_fast(int k, int ni, const PassArgs& a, unsigned grid, size_t lds, hipStream_t s);
// forward / adjoint pass of complex64 radix-8 digits, general tiles
hipError_t launch_cpass8(const PassArgs& a, unsigned grid, size_t lds, hipStream_t s);
hipError_t launch_cbwd8_fast(int k, int ni, const CBwdArgs& a, unsigned grid, size_t lds, hipStream_t s);

// k dominant coefficients of every instance (ascending indices, ties to the
// lower index); with recon != NULL also the zero-filled sparse coefficient
// vector (the caller then applies the inverse transform in place)
// (few large instances: many work-groups per instance, with `meta` bytes
// of workspace from topk_meta_bytes; otherwise one work-group per instance)
hipError_t launch_topk(DT dt, const void* coef, int64_t N, int64_t batch, int64_t k, int64_t* idx, void* val,
                       void* recon, void* meta, hipStream_t s);
size_t topk_meta_bytes(int64_t N, int64_t batch);

// elementwise storage conversion bf16/f16 <-> float32 (RNE to 16 bits)
hipError_t launch_convert(DT from, DT to, const void* in, void* out, int64_t n, hipStream_t s);

struct RaggedArgs;
// ragged-batch launch (all phases with grid barriers, or one phase)
hipError_t launch_ragged(DT dt, const RaggedArgs& a, unsigned grid, size_t lds, hipStream_t s);
// the items [phase_start[0], phase_start[1]) of one item class
hipError_t launch_ragged_cls(DT dt, int cls, const RaggedArgs& a, unsigned grid, size_t lds, hipStream_t s);
// co-resident work-groups per compute unit of the ragged kernel
hipError_t ragged_occupancy(DT dt, size_t lds, int* blocks_per_cu);

}  // namespace gtt
