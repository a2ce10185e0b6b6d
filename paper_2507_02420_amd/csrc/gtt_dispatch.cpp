// Dtype dispatch to the per-dtype kernel translation units.
#include <map>
#include <mutex>
#include <tuple>

#include "gtt_launch.hpp"

namespace gtt {

hipError_t launch_pass_f64(int, int, const PassArgs&, unsigned, size_t, hipStream_t);
hipError_t launch_pass_f32(int, int, const PassArgs&, unsigned, size_t, hipStream_t);
hipError_t launch_pass_c128(int, int, const PassArgs&, unsigned, size_t, hipStream_t);
hipError_t launch_pass_c64(int, int, const PassArgs&, unsigned, size_t, hipStream_t);
hipError_t launch_pass_bf16(int, int, const PassArgs&, unsigned, size_t, hipStream_t);
hipError_t launch_pass_f16(int, int, const PassArgs&, unsigned, size_t, hipStream_t);
hipError_t launch_pass_i32(int, int, const PassArgs&, unsigned, size_t, hipStream_t);

hipError_t launch_bwd_f64(const BwdArgs&, int, int, unsigned, int, size_t, hipStream_t);
int launch_bwd_threads_f64(int, size_t);
int bwd_block_digits_f64(int);
hipError_t launch_bwd_f32(const BwdArgs&, int, int, unsigned, int, size_t, hipStream_t);
int launch_bwd_threads_f32(int, size_t);
int bwd_block_digits_f32(int);
hipError_t launch_bwd_c128(const BwdArgs&, int, int, unsigned, int, size_t, hipStream_t);
int launch_bwd_threads_c128(int, size_t);
int bwd_block_digits_c128(int);
hipError_t launch_bwd_c64(const BwdArgs&, int, int, unsigned, int, size_t, hipStream_t);
int launch_bwd_threads_c64(int, size_t);
int bwd_block_digits_c64(int);
hipError_t launch_bwd_bf16(const BwdArgs&, int, int, unsigned, int, size_t, hipStream_t);
int launch_bwd_threads_bf16(int, size_t);
int bwd_block_digits_bf16(int);
hipError_t launch_bwd_f16(const BwdArgs&, int, int, unsigned, int, size_t, hipStream_t);
int launch_bwd_threads_f16(int, size_t);
int bwd_block_digits_f16(int);
hipError_t launch_reduce_f64(const void*, int64_t, int, void*, hipStream_t);
hipError_t launch_reduce_f32(const void*, int64_t, int, void*, hipStream_t);
hipError_t launch_reduce_c128(const void*, int64_t, int, void*, hipStream_t);
hipError_t launch_reduce_c64(const void*, int64_t, int, void*, hipStream_t);
hipError_t launch_reduce_bf16(const void*, int64_t, int, void*, hipStream_t);
hipError_t launch_reduce_f16(const void*, int64_t, int, void*, hipStream_t);

int bwd_block_digits(DT dt, int b) {
    switch (dt) {
        case DT::F64: return bwd_block_digits_f64(b);
        case DT::F32: return bwd_block_digits_f32(b);
        case DT::C128: return bwd_block_digits_c128(b);
        case DT::C64: return bwd_block_digits_c64(b);
        case DT::BF16: return bwd_block_digits_bf16(b);
        case DT::F16: return bwd_block_digits_f16(b);
        default: return 0;
    }
}

hipError_t launch_bwd(DT dt, const BwdArgs& a, int maxb, int radix, unsigned grid, int threads, size_t lds,
                      hipStream_t s) {
    switch (dt) {
        case DT::F64: return launch_bwd_f64(a, maxb, radix, grid, threads, lds, s);
        case DT::F32: return launch_bwd_f32(a, maxb, radix, grid, threads, lds, s);
        case DT::C128: return launch_bwd_c128(a, maxb, radix, grid, threads, lds, s);
        case DT::C64: return launch_bwd_c64(a, maxb, radix, grid, threads, lds, s);
        case DT::BF16: return launch_bwd_bf16(a, maxb, radix, grid, threads, lds, s);
        case DT::F16: return launch_bwd_f16(a, maxb, radix, grid, threads, lds, s);
        default: return hipErrorInvalidValue;
    }
}

int launch_bwd_threads(DT dt, int radix, size_t lds) {
    if (radix <= 0) return kThreads;
    // occupancy queries once per (device, dtype, radix, LDS bytes)
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, size_t>, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = -1;
    const auto key = std::make_tuple(dev, (int)dt, radix, lds);
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    int nt = kThreads;
    switch (dt) {
        case DT::F64: nt = launch_bwd_threads_f64(radix, lds); break;
        case DT::F32: nt = launch_bwd_threads_f32(radix, lds); break;
        case DT::C128: nt = launch_bwd_threads_c128(radix, lds); break;
        case DT::C64: nt = launch_bwd_threads_c64(radix, lds); break;
        case DT::BF16: nt = launch_bwd_threads_bf16(radix, lds); break;
        case DT::F16: nt = launch_bwd_threads_f16(radix, lds); break;
        default: break;
    }
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = nt;
    return nt;
}

hipError_t launch_reduce(DT dt, const void* partials, int64_t nparts, int bb, void* out, hipStream_t s) {
    switch (dt) {
        case DT::F64: return launch_reduce_f64(partials, nparts, bb, out, s);
        case DT::F32: return launch_reduce_f32(partials, nparts, bb, out, s);
        case DT::C128: return launch_reduce_c128(partials, nparts, bb, out, s);
        case DT::C64: return launch_reduce_c64(partials, nparts, bb, out, s);
        case DT::BF16: return launch_reduce_bf16(partials, nparts, bb, out, s);
        case DT::F16: return launch_reduce_f16(partials, nparts, bb, out, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_ragged_f64(const RaggedArgs&, unsigned, size_t, hipStream_t);
hipError_t ragged_occupancy_f64(size_t, int*);
hipError_t launch_ragged_f32(const RaggedArgs&, unsigned, size_t, hipStream_t);
hipError_t ragged_occupancy_f32(size_t, int*);
hipError_t launch_ragged_c128(const RaggedArgs&, unsigned, size_t, hipStream_t);
hipError_t ragged_occupancy_c128(size_t, int*);
hipError_t launch_ragged_c64(const RaggedArgs&, unsigned, size_t, hipStream_t);
hipError_t ragged_occupancy_c64(size_t, int*);
hipError_t launch_ragged_bf16(const RaggedArgs&, unsigned, size_t, hipStream_t);
hipError_t ragged_occupancy_bf16(size_t, int*);
hipError_t launch_ragged_f16(const RaggedArgs&, unsigned, size_t, hipStream_t);
hipError_t ragged_occupancy_f16(size_t, int*);
hipError_t launch_ragged_i32(const RaggedArgs&, unsigned, size_t, hipStream_t);
hipError_t ragged_occupancy_i32(size_t, int*);

hipError_t launch_ragged_cls_f64(int, const RaggedArgs&, unsigned, size_t, hipStream_t);
hipError_t launch_ragged_cls_f32(int, const RaggedArgs&, unsigned, size_t, hipStream_t);
hipError_t launch_ragged_cls_c128(int, const RaggedArgs&, unsigned, size_t, hipStream_t);
hipError_t launch_ragged_cls_c64(int, const RaggedArgs&, unsigned, size_t, hipStream_t);
hipError_t launch_ragged_cls_bf16(int, const RaggedArgs&, unsigned, size_t, hipStream_t);
hipError_t launch_ragged_cls_f16(int, const RaggedArgs&, unsigned, size_t, hipStream_t);
hipError_t launch_ragged_cls_i32(int, const RaggedArgs&, unsigned, size_t, hipStream_t);

hipError_t launch_ragged_cls(DT dt, int cls, const RaggedArgs& a, unsigned grid, size_t lds, hipStream_t s) {
    switch (dt) {
        case DT::F64: return launch_ragged_cls_f64(cls, a, grid, lds, s);
        case DT::F32: return launch_ragged_cls_f32(cls, a, grid, lds, s);
        case DT::C128: return launch_ragged_cls_c128(cls, a, grid, lds, s);
        case DT::C64: return launch_ragged_cls_c64(cls, a, grid, lds, s);
        case DT::BF16: return launch_ragged_cls_bf16(cls, a, grid, lds, s);
        case DT::F16: return launch_ragged_cls_f16(cls, a, grid, lds, s);
        case DT::I32: return launch_ragged_cls_i32(cls, a, grid, lds, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_ragged(DT dt, const RaggedArgs& a, unsigned grid, size_t lds, hipStream_t s) {
    switch (dt) {
        case DT::F64: return launch_ragged_f64(a, grid, lds, s);
        case DT::F32: return launch_ragged_f32(a, grid, lds, s);
        case DT::C128: return launch_ragged_c128(a, grid, lds, s);
        case DT::C64: return launch_ragged_c64(a, grid, lds, s);
        case DT::BF16: return launch_ragged_bf16(a, grid, lds, s);
        case DT::F16: return launch_ragged_f16(a, grid, lds, s);
        case DT::I32: return launch_ragged_i32(a, grid, lds, s);
    }
    return hipErrorInvalidValue;
}

hipError_t ragged_occupancy(DT dt, size_t lds, int* b) {
    switch (dt) {
        case DT::F64: return ragged_occupancy_f64(lds, b);
        case DT::F32: return ragged_occupancy_f32(lds, b);
        case DT::C128: return ragged_occupancy_c128(lds, b);
        case DT::C64: return ragged_occupancy_c64(lds, b);
        case DT::BF16: return ragged_occupancy_bf16(lds, b);
        case DT::F16: return ragged_occupancy_f16(lds, b);
        case DT::I32: return ragged_occupancy_i32(lds, b);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_pass(DT dt, int b, int kind, const PassArgs& a, unsigned grid, size_t lds, hipStream_t s) {
    switch (dt) {
        case DT::F64: return launch_pass_f64(b, kind, a, grid, lds, s);
        case DT::F32: return launch_pass_f32(b, kind, a, grid, lds, s);
        case DT::C128: return launch_pass_c128(b, kind, a, grid, lds, s);
        case DT::C64: return launch_pass_c64(b, kind, a, grid, lds, s);
        case DT::BF16: return launch_pass_bf16(b, kind, a, grid, lds, s);
        case DT::F16: return launch_pass_f16(b, kind, a, grid, lds, s);
        case DT::I32: return launch_pass_i32(b, kind, a, grid, lds, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace gtt
