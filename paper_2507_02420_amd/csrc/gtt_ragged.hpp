// Ragged batches: instances of different radix and length (each its own GTT,
// Def. 2.4) packed in one buffer.  The host lays out a device work list of
// (descriptor, tile) items, one descriptor per (instance, digit group);
// phase p holds the tiles of digit group p of every instance, sorted by item
// class (VALU radix 2..5, runtime radix, matrix-core radix 16 / 32).
//
// Per-phase mode (the default) launches one kernel per run of one class in a
// phase, specialised to that class: VALU and runtime-radix classes take one
// tile per work-group; matrix-core classes loop over their items on a
// resident grid, keeping W's fragments while consecutive items share W.
//
// Persistent mode runs every phase in ONE launch of the all-class kernel (a
// work-group takes the items of the current phase round-robin and dispatches
// on the class) and separates the phases by a grid barrier (the next digit
// group of an instance needs all tiles of the previous one).  The barrier
// counts arrivals with a device-scope atomic; the last work-group to arrive
// resets the count and advances a generation word the others wait on, so the
// state returns to zero after every barrier and the launch can be replayed
// from a captured graph.  The grid never exceeds the number of co-resident
// work-groups (occupancy x compute units, not a cooperative launch), and
// every wait is bounded: after `spin_limit` polls a work-group raises the
// failure word; every work-group that sees it leaves the kernel at its next
// barrier (no wave can hang, no phase runs on partial data).  A one-thread
// kernel before every persistent launch zeroes the arrival and generation
// words and moves a raised failure word into a sticky record that the host
// reads and clears with gtt_plan_check.
#pragma once

#include "gtt_args.hpp"
#include "gtt_mfma.hpp"
#include "gtt_pass.hpp"
#include "gtt_types.hpp"

namespace gtt {

struct RaggedDesc {
    PassArgs a;          // tile geometry of this (instance, group)
    int64_t in_off;      // element offset of the group's input
    int64_t out_off;     // element offset of the group's output
    int64_t mid_off_saved;  // offset of this group's output inside `saved`
    int64_t w_off;       // element offset of the instance's W in the W table
    int32_t in_sel;      // 0: x, 1: y, 2: intermediate (saved if given, else y)
    int32_t out_sel;     // 1: y, 2: intermediate
    int32_t in_mid_saved;// 1 when in_sel == 2 (offset in saved is in_off_saved)
    int32_t b;
    int32_t kind;        // kKindValu / kKindGeneric / kKindMfma
    int32_t pad0;
    int64_t in_off_saved;
};

struct RaggedItem {
    int32_t d;           // descriptor index
    int32_t pad0;
    int64_t tile;        // tile index within the descriptor's group
};

constexpr int kMaxPhases = 8;

struct RaggedArgs {
    const RaggedDesc* desc;
    const RaggedItem* items;
    int64_t phase_start[kMaxPhases + 1];
    int32_t nphases;
    int32_t persistent;  // 1: all phases in this launch, grid barriers between
    int32_t phase;       // phase of a per-phase launch
    int32_t adjoint;
    const void* x;
    void* y;
    void* saved;
    const void* W;
    unsigned* bar;       // [0] arrivals, [1] generation, [2] failure of this
                         // launch, [3] sticky failure record
    uint32_t spin_limit; // polls of a barrier wait before it gives up
};

// Returns false when the barrier failed (this or another work-group gave up
// waiting); the caller then leaves the kernel.
__device__ __forceinline__ bool grid_barrier(unsigned* bar, unsigned nblocks, uint32_t spin_limit) {
    __shared__ unsigned failed;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned gen = __hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        __atomic_thread_fence(__ATOMIC_RELEASE);  // this block's tile stores
        const unsigned arrived =
            __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == nblocks - 1) {
            __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            // bounded wait (the default limit, 2^24 polls with s_sleep, is
            // several seconds); a failure raised elsewhere ends it at once
            // (a limit of 0 gives up without polling)
            for (uint32_t spin = 0;; ++spin) {
                if (spin >= spin_limit || __hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    __hip_atomic_store(&bar[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                if (__hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != gen) break;
                __builtin_amdgcn_s_sleep(4);
            }
        }
        __atomic_thread_fence(__ATOMIC_ACQUIRE);
        failed = __hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    return failed == 0;
}

template <typename C, int B>
__device__ __forceinline__ void load_w_ptr(C (&w)[B * B], const C* __restrict__ Wg, int adjoint, C* wl) {
    if constexpr (B * B * sizeof(C) <= 128) {
#pragma unroll
        for (int r = 0; r < B; ++r)
#pragma unroll
            for (int q = 0; q < B; ++q) w[r * B + q] = adjoint ? cconj(Wg[q * B + r]) : Wg[r * B + q];
    } else {
        for (int e = threadIdx.x; e < B * B; e += kThreads) {
            const int r = e / B, q = e % B;
            wl[e] = adjoint ? cconj(Wg[q * B + r]) : Wg[e];
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < B * B; ++e) w[e] = wl[e];
    }
}

template <typename T, int B>
__device__ __forceinline__ void ragged_tile_valu(unsigned char* smem, const PassArgs& a, const T* in, T* out,
                                              const typename Tr<T>::C* W, int adjoint, int64_t t) {
    using C = typename Tr<T>::C;
    constexpr int RD = RegDigits<B>::v;
    C* wl = reinterpret_cast<C*>(smem);
    C* lds = wl + 64;  // first 64 elements: staging for W (radix <= 8)
    C w[B * B];
    load_w_ptr<C, B>(w, W, adjoint, wl);
    const uint32_t rows = (uint32_t)a.P * (uint32_t)a.G;
    tile_load<T, C>(lds, a, in, t, rows);
    __syncthreads();
    run_stages<C, B, RD>(lds, a, rows, w);
    tile_store<T, C>(lds, a, out, t, rows);
    __syncthreads();
}

template <typename T>
__device__ __forceinline__ void ragged_tile_generic(unsigned char* smem, const PassArgs& a, const T* in, T* out,
                                                 const typename Tr<T>::C* W, int adjoint, int64_t t) {
    using C = typename Tr<T>::C;
    C* Wl = reinterpret_cast<C*>(smem);
    const uint32_t rows = (uint32_t)a.P * (uint32_t)a.G;
    const uint32_t tileE = rows << a.logC;
    const uint32_t wpad = ((uint32_t)a.wtotal + 15u) & ~15u;
    C* buf0 = Wl + wpad;
    C* buf1 = buf0 + lds_tile_elems(tileE, a.pad_shift);  // only for radices above 16
    for (int j = 0, done = 0; j < a.k; ++j) {
        const int bj = a.rad[j];
        for (int e = threadIdx.x; e < bj * bj; e += kThreads) {
            const int r = e / bj, q = e - r * bj;
            Wl[done + e] = adjoint ? cconj(W[a.wofs[j] + q * bj + r]) : W[a.wofs[j] + e];
        }
        done += bj * bj;
    }
    tile_load<T, C>(buf0, a, in, t, rows);
    __syncthreads();
    const C* res = generic_digits<C>(buf0, buf1, Wl, a, rows);
    tile_store<T, C>(res, a, out, t, rows);
    __syncthreads();
}

// Item classes.  The per-phase launches run the items of one class with a
// kernel specialised to it (its own registers and LDS, hence occupancy);
// the persistent launch dispatches every item at run time.
constexpr int kClsAny = -1;
constexpr int kClsGeneric = 0;  // 2..5: VALU radix; 16, 32: matrix-core radix

__host__ __device__ inline int ragged_class(int kind, int b) {
    if (kind == kKindValu) return (b >= 2 && b <= 5) ? b : kClsGeneric;
    if (kind == kKindMfma) return b;
    return kClsGeneric;
}

// input and output of an item's group (x / y / the saved intermediates)
template <typename T>
__device__ __forceinline__ const T* ragged_in(const RaggedArgs& r, const RaggedDesc& d) {
    if (d.in_sel == 0) return static_cast<const T*>(r.x) + d.in_off;
    if (d.in_sel == 1 || !r.saved) return static_cast<const T*>(r.y) + d.in_off;
    return static_cast<const T*>(r.saved) + d.in_off_saved;
}
template <typename T>
__device__ __forceinline__ T* ragged_out(const RaggedArgs& r, const RaggedDesc& d) {
    if (d.out_sel == 1 || !r.saved) return static_cast<T*>(r.y) + d.out_off;
    return static_cast<T*>(r.saved) + d.mid_off_saved;
}

template <typename T, int CLS>
__device__ __forceinline__ void ragged_item(unsigned char* smem, const RaggedArgs& r, const RaggedItem& it) {
    using C = typename Tr<T>::C;
    const RaggedDesc& d = r.desc[it.d];
    const T* in = ragged_in<T>(r, d);
    T* out = ragged_out<T>(r, d);
    const C* W = static_cast<const C*>(r.W) + d.w_off;
    if constexpr (CLS == kClsAny) {
        if (d.kind == kKindValu) {
            switch (d.b) {
                case 2: ragged_tile_valu<T, 2>(smem, d.a, in, out, W, r.adjoint, it.tile); break;
                case 3: ragged_tile_valu<T, 3>(smem, d.a, in, out, W, r.adjoint, it.tile); break;
                case 4: ragged_tile_valu<T, 4>(smem, d.a, in, out, W, r.adjoint, it.tile); break;
                case 5: ragged_tile_valu<T, 5>(smem, d.a, in, out, W, r.adjoint, it.tile); break;
                default: ragged_tile_generic<T>(smem, d.a, in, out, W, r.adjoint, it.tile); break;
            }
        } else {
            ragged_tile_generic<T>(smem, d.a, in, out, W, r.adjoint, it.tile);
        }
    } else if constexpr (CLS == kClsGeneric) {
        ragged_tile_generic<T>(smem, d.a, in, out, W, r.adjoint, it.tile);
    } else if constexpr (CLS <= 5) {
        ragged_tile_valu<T, CLS>(smem, d.a, in, out, W, r.adjoint, it.tile);
    } else {
        static_assert(CLS <= 5, "matrix-core classes run ragged_mfma_items");
    }
}

template <typename T, int B>
__device__ __forceinline__ void ragged_tile_mfma_wf(unsigned char* smem, const PassArgs& a, const T* in, T* out,
                                                    const WFrag<T, B>& wf, int64_t t) {
    const uint32_t rows = (uint32_t)a.P * (uint32_t)a.G;
    if constexpr (std::is_same<T, float>::value) {
        float* lds = reinterpret_cast<float*>(smem + 256);
        tile_load<T, float>(lds, a, in, t, rows);
        __syncthreads();
        for (int j = 0; j < a.k; ++j) {
            mfma_stage<T, B>(lds, a, j, rows, wf);
            __syncthreads();
        }
        tile_store<T, float>(lds, a, out, t, rows);
    } else {
        uint16_t* lds = reinterpret_cast<uint16_t*>(smem + 256);
        tile_load16<T>(lds, a, in, t, rows);
        __syncthreads();
        for (int j = 0; j < a.k; ++j) {
            mfma_stage16<T, B>(lds, a, j, rows, wf);
            __syncthreads();
        }
        tile_store16<T>(lds, a, out, t, rows);
    }
    __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(kThreads) void gtt_ragged_kernel(RaggedArgs r) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr bool kMfma = sizeof(T) == 2 || std::is_same<T, float>::value;
    const int p0 = r.persistent ? 0 : r.phase;
    const int p1 = r.persistent ? r.nphases : r.phase + 1;
    // matrix-core items keep W's fragments while consecutive items share W
    [[maybe_unused]] typename std::conditional<kMfma, WFrag<T, 16>, char>::type wf16;
    [[maybe_unused]] typename std::conditional<kMfma, WFrag<T, 32>, char>::type wf32;
    [[maybe_unused]] int64_t w16 = -1, w32 = -1;
    for (int p = p0; p < p1; ++p) {
        for (int64_t i = r.phase_start[p] + blockIdx.x; i < r.phase_start[p + 1]; i += gridDim.x) {
            const RaggedItem it = r.items[i];
            if constexpr (kMfma) {
                const RaggedDesc& d = r.desc[it.d];
                if (d.kind == kKindMfma) {
                    PassArgs aw;  // only W / adjoint are read by the fragment loader
                    aw.W = static_cast<const float*>(r.W) + d.w_off;
                    aw.adjoint = r.adjoint;
                    if (d.b == 16) {
                        if (d.w_off != w16) {
                            load_w_frag<T, 16>(wf16, aw);
                            w16 = d.w_off;
                        }
                        ragged_tile_mfma_wf<T, 16>(smem_raw, d.a, ragged_in<T>(r, d), ragged_out<T>(r, d), wf16, it.tile);
                    } else {
                        if (d.w_off != w32) {
                            load_w_frag<T, 32>(wf32, aw);
                            w32 = d.w_off;
                        }
                        ragged_tile_mfma_wf<T, 32>(smem_raw, d.a, ragged_in<T>(r, d), ragged_out<T>(r, d), wf32, it.tile);
                    }
                    continue;
                }
            }
            ragged_item<T, kClsAny>(smem_raw, r, it);
        }
        if (r.persistent && p + 1 < p1 && !grid_barrier(r.bar, gridDim.x, r.spin_limit)) return;
    }
}

// Matrix-core items (one class, one phase): the work-groups loop over the
// items and keep W's fragments while consecutive items share W.  (A
// register prefetch of the next item, as in the uniform pass, lowers the
// occupancy of these kernels and was slower.)
template <typename T, int B>
__device__ __forceinline__ void ragged_mfma_items(unsigned char* smem, const RaggedArgs& r) {
    constexpr bool k16 = sizeof(T) == 2;
    using L = typename std::conditional<k16, uint16_t, float>::type;
    L* lds = reinterpret_cast<L*>(smem + 256);
    WFrag<T, B> wf;
    int64_t wcur = -1;
    for (int64_t i = r.phase_start[0] + blockIdx.x; i < r.phase_start[1]; i += gridDim.x) {
        const RaggedItem it = r.items[i];
        const RaggedDesc& d = r.desc[it.d];
        const PassArgs& a = d.a;
        if (d.w_off != wcur) {
            PassArgs aw;  // only W / adjoint are read by the fragment loader
            aw.W = static_cast<const float*>(r.W) + d.w_off;
            aw.adjoint = r.adjoint;
            load_w_frag<T, B>(wf, aw);
            wcur = d.w_off;
        }
        const uint32_t rows = (uint32_t)a.P * (uint32_t)a.G;
        if constexpr (k16)
            tile_load16<T>(lds, a, ragged_in<T>(r, d), it.tile, rows);
        else
            tile_load<T, float>(lds, a, ragged_in<T>(r, d), it.tile, rows);
        __syncthreads();
        for (int j = 0; j < a.k; ++j) {
            if constexpr (k16)
                mfma_stage16<T, B>(lds, a, j, rows, wf);
            else
                mfma_stage<T, B>(lds, a, j, rows, wf);
            __syncthreads();
        }
        if constexpr (k16)
            tile_store16<T>(lds, a, ragged_out<T>(r, d), it.tile, rows);
        else
            tile_store<T, float>(lds, a, ragged_out<T>(r, d), it.tile, rows);
        __syncthreads();
    }
}

// The items [phase_start[0], phase_start[1]) of one class.
template <typename T, int CLS>
__global__ __launch_bounds__(kThreads) void gtt_ragged_class_kernel(RaggedArgs r) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    if constexpr (CLS >= 16) {
        static_assert(sizeof(T) == 2 || std::is_same<T, float>::value,
                      "matrix-core item classes exist for 16-bit and float storage only");
        ragged_mfma_items<T, CLS>(smem_raw, r);
    } else {
        for (int64_t i = r.phase_start[0] + blockIdx.x; i < r.phase_start[1]; i += gridDim.x)
            ragged_item<T, CLS>(smem_raw, r, r.items[i]);
    }
}

}  // namespace gtt
