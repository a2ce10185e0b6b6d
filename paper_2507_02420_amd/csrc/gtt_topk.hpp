// Selection of the k dominant coefficients of every instance (the classical
// state-transmission protocol of §4.1.1: transform, keep the k coefficients of
// largest magnitude, send their indices and values, invert).
//
// One work-group per instance.  The magnitude |c|^2 (|c| for int32) is mapped
// to an unsigned key whose order is the order of the magnitudes (IEEE bits of
// a non-negative number).  A most-significant-digit radix select (8 bits per
// sweep, LDS histogram) finds the k-th largest key t and how many elements
// equal to t must be taken; an ordered compaction then writes, in ascending
// index order, every element with key > t and the lowest-indexed elements
// with key == t.  Ties are therefore broken towards the lower index.
#pragma once

#include "gtt_args.hpp"
#include "gtt_types.hpp"

namespace gtt {

constexpr int kTopkThreads = 1024;

template <typename T>
struct TopkKey {
    using K = uint32_t;
};
template <>
struct TopkKey<double> {
    using K = uint64_t;
};
template <>
struct TopkKey<cd> {
    using K = uint64_t;
};

__device__ __forceinline__ uint32_t topk_key(float v) { const float m = v * v; return __float_as_uint(m); }
__device__ __forceinline__ uint32_t topk_key(bf16 v) { return topk_key(to_c(v)); }
__device__ __forceinline__ uint32_t topk_key(f16 v) { return topk_key(to_c(v)); }
__device__ __forceinline__ uint32_t topk_key(cf v) {
    const float m = __builtin_fmaf(v.re, v.re, v.im * v.im);
    return __float_as_uint(m);
}
__device__ __forceinline__ uint32_t topk_key(int32_t v) {
    return v < 0 ? (uint32_t)0u - (uint32_t)v : (uint32_t)v;
}
__device__ __forceinline__ uint64_t topk_key(double v) { return (uint64_t)__double_as_longlong(v * v); }
__device__ __forceinline__ uint64_t topk_key(cd v) {
    return (uint64_t)__double_as_longlong(__builtin_fma(v.re, v.re, v.im * v.im));
}

// exclusive prefix count of flag over the work-group (in thread order) and
// the total; wsum: kTopkThreads/64 ints of LDS
__device__ __forceinline__ uint32_t block_excl_count(bool flag, uint32_t* wsum, uint32_t* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t m = __ballot(flag);
    const uint32_t below = (uint32_t)__popcll(m & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
    if (lane == 0) wsum[wave] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t before = 0, tot = 0;
    for (int w = 0; w < kTopkThreads / 64; ++w) {
        const uint32_t c = wsum[w];
        if (w < wave) before += c;
        tot += c;
    }
    __syncthreads();
    *total = tot;
    return before + below;
}

template <typename T>
__global__ __launch_bounds__(kTopkThreads) void gtt_topk_kernel(const T* __restrict__ coef, int64_t N, int64_t k,
                                                                 int64_t* __restrict__ idx, T* __restrict__ val) {
    using K = typename TopkKey<T>::K;
    constexpr int KB = 8 * sizeof(K);
    __shared__ uint32_t hist[256];
    __shared__ uint32_t wsum[kTopkThreads / 64];
    __shared__ K s_prefix;
    __shared__ int64_t s_remaining;
    const T* c = coef + (int64_t)blockIdx.x * N;
    int64_t* oi = idx + (int64_t)blockIdx.x * k;
    T* ov = val + (int64_t)blockIdx.x * k;
    K prefix = 0, pmask = 0;
    int64_t remaining = k;
    for (int shift = KB - 8; shift >= 0; shift -= 8) {
        for (int d = threadIdx.x; d < 256; d += kTopkThreads) hist[d] = 0;
        __syncthreads();
        for (int64_t i = threadIdx.x; i < N; i += kTopkThreads) {
            const K key = topk_key(c[i]);
            if ((key & pmask) == prefix) atomicAdd(&hist[(uint32_t)(key >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t cum = 0;
            int sel = 0;
            for (int d = 255; d >= 0; --d) {
                if (cum + (int64_t)hist[d] >= remaining) {
                    sel = d;
                    break;
                }
                cum += hist[d];
            }
            s_prefix = prefix | ((K)sel << shift);
            s_remaining = remaining - cum;
        }
        __syncthreads();
        prefix = s_prefix;
        remaining = s_remaining;
        pmask |= ((K)255 << shift);
        __syncthreads();
    }
    // prefix is the k-th largest key; `remaining` elements equal to it are taken
    const K thr = prefix;
    const int64_t need_eq = remaining;
    int64_t eq_seen = 0, out_seen = 0;
    for (int64_t base = 0; base < N; base += kTopkThreads) {
        const int64_t i = base + threadIdx.x;
        K key = 0;
        bool in = i < N;
        if (in) key = topk_key(c[i]);
        const bool gt = in && key > thr;
        const bool eq = in && key == thr;
        uint32_t eq_tot;
        const uint32_t eq_rank = block_excl_count(eq, wsum, &eq_tot);
        const bool take = gt || (eq && eq_seen + (int64_t)eq_rank < need_eq);
        uint32_t take_tot;
        const uint32_t pos = block_excl_count(take, wsum, &take_tot);
        if (take) {
            oi[out_seen + pos] = i;
            ov[out_seen + pos] = c[i];
        }
        eq_seen += eq_tot;
        out_seen += take_tot;
        if (out_seen >= k) break;  // uniform: every thread sees the same totals
    }
}

// recon[inst][idx[inst][j]] = val[inst][j] over a zeroed buffer
template <typename T>
__global__ __launch_bounds__(256) void gtt_scatter_kernel(T* __restrict__ out, int64_t N, int64_t k, int64_t batch,
                                                          const int64_t* __restrict__ idx,
                                                          const T* __restrict__ val) {
    const int64_t n = batch * k;
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256) {
        const int64_t inst = j / k;
        out[inst * N + idx[j]] = val[j];
    }
}

template <typename T>
__global__ __launch_bounds__(256) void gtt_zero_kernel(T* __restrict__ out, int64_t n) {
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256)
        out[j] = from_c<T>(czero<typename Tr<T>::C>());
}

}  // namespace gtt
