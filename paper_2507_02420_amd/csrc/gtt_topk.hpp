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

// exclusive prefix count of flag over the work-group of NT threads (in
// thread order) and the total; wsum: NT/64 ints of LDS
template <int NT = kTopkThreads>
__device__ __forceinline__ uint32_t block_excl_count(bool flag, uint32_t* wsum, uint32_t* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t m = __ballot(flag);
    const uint32_t below = (uint32_t)__popcll(m & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
    if (lane == 0) wsum[wave] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t before = 0, tot = 0;
    for (int w = 0; w < NT / 64; ++w) {
        const uint32_t c = wsum[w];
        if (w < wave) before += c;
        tot += c;
    }
    __syncthreads();
    *total = tot;
    return before + below;
}

// The digit of the k-th largest key: the largest digit value d whose count
// of keys with digit >= d reaches the keys still to be taken.  Thread
// i < 256 of the work-group holds the count hv of digit 255 - i, so an
// inclusive scan over those threads gives every digit's count from the top
// (P) and the count strictly above it (P - hv); the one thread where P
// first reaches `remaining` returns true with the digit and the count above
// it.  Fewer keys than still wanted (not possible for k <= N) take digit 0
// and everything above it.  Every thread of the work-group calls it (it
// holds work-group barriers); sc: 2 x 256 words of LDS.
__device__ __forceinline__ bool topk_digit_choice(uint64_t hv, int64_t remaining, uint64_t (*sc)[256], int* sel,
                                                  int64_t* cum) {
    const int i = threadIdx.x;
    if (i < 256) sc[0][i] = hv;
    __syncthreads();
    int cur = 0;
    for (int o = 1; o < 256; o <<= 1) {
        if (i < 256) {
            uint64_t v = sc[cur][i];
            if (i >= o) v += sc[cur][i - o];
            sc[cur ^ 1][i] = v;
        }
        cur ^= 1;
        __syncthreads();
    }
    if (i >= 256) return false;
    const int64_t P = (int64_t)sc[cur][i], above = P - (int64_t)hv;
    if (P >= remaining && (i == 0 || above < remaining)) {
        *sel = 255 - i;
        *cum = above;
        return true;
    }
    if (i == 255 && P < remaining) {
        *sel = 0;
        *cum = P;
        return true;
    }
    return false;
}

template <typename T>
__global__ __launch_bounds__(kTopkThreads) void gtt_topk_kernel(const T* __restrict__ coef, int64_t N, int64_t k,
                                                                 int64_t* __restrict__ idx, T* __restrict__ val) {
    using K = typename TopkKey<T>::K;
    constexpr int KB = 8 * sizeof(K);
    __shared__ uint32_t hist[256];
    __shared__ uint32_t wsum[kTopkThreads / 64];
    __shared__ uint64_t sc[2][256];
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
        int sel;
        int64_t cum;
        if (topk_digit_choice(threadIdx.x < 256 ? hist[255 - threadIdx.x] : 0u, remaining, sc, &sel, &cum)) {
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
        const uint32_t eq_rank = block_excl_count<>(eq, wsum, &eq_tot);
        const bool take = gt || (eq && eq_seen + (int64_t)eq_rank < need_eq);
        uint32_t take_tot;
        const uint32_t pos = block_excl_count<>(take, wsum, &take_tot);
        if (take) {
            oi[out_seen + pos] = i;
            ov[out_seen + pos] = c[i];
        }
        eq_seen += eq_tot;
        out_seen += take_tot;
        if (out_seen >= k) break;  // uniform: every thread sees the same totals
    }
}

// ---------------------------------------------------------------------------
// The same selection spread over many work-groups per instance (few large
// instances: one work-group each would leave most compute units idle).  An
// instance is cut into chunks of kTopkChunk elements, one work-group each:
//   per 8-bit digit of the key (most significant first): every chunk adds its
//   histogram of the keys that match the prefix chosen so far into the
//   instance's global histogram (atomics), then one work-group per instance
//   picks the digit holding the k-th largest key and clears the histogram;
//   ordered compaction: every chunk counts its keys above and equal to the
//   threshold, one work-group per instance turns the counts into each
//   chunk's output offset (chunks in index order: the elements above the
//   threshold before the chunk, plus min(equal elements before it, equal
//   elements needed)), and every chunk writes its elements in index order.
// The state, histograms and per-chunk counts live in the caller's workspace.
// ---------------------------------------------------------------------------
constexpr int kTopkChunkThreads = 256;
constexpr int kTopkChunk = kTopkChunkThreads * 16;

struct TopkState {
    uint64_t prefix, pmask;
    int64_t remaining;
    int64_t pad;
};

template <typename K>
__global__ __launch_bounds__(256) void gtt_topk_init_kernel(TopkState* st, uint32_t* ghist, int64_t batch, int64_t k) {
    const int64_t t = blockIdx.x;
    if (t >= batch) return;
    if (threadIdx.x == 0) st[t] = TopkState{0, 0, k, 0};
    ghist[t * 256 + threadIdx.x] = 0u;
}

template <typename T>
__global__ __launch_bounds__(kTopkChunkThreads) void gtt_topk_hist_kernel(const T* __restrict__ coef, int64_t N,
                                                                          const TopkState* __restrict__ st,
                                                                          uint32_t* __restrict__ ghist, int shift) {
    using K = typename TopkKey<T>::K;
    __shared__ uint32_t hist[256];
    const int64_t t = blockIdx.y;
    const int64_t c0 = (int64_t)blockIdx.x * kTopkChunk;
    const int64_t c1 = c0 + kTopkChunk < N ? c0 + kTopkChunk : N;
    hist[threadIdx.x] = 0u;
    __syncthreads();
    const K prefix = (K)st[t].prefix, pmask = (K)st[t].pmask;
    const T* c = coef + t * N;
    for (int64_t i = c0 + threadIdx.x; i < c1; i += kTopkChunkThreads) {
        const K key = topk_key(c[i]);
        if ((key & pmask) == prefix) atomicAdd(&hist[(uint32_t)(key >> shift) & 255u], 1u);
    }
    __syncthreads();
    const uint32_t h = hist[threadIdx.x];
    if (h) atomicAdd(&ghist[t * 256 + threadIdx.x], h);
}

// the digit choice of one instance from its global histogram (cleared for
// the next digit on the way)
template <typename K>
__global__ __launch_bounds__(256) void gtt_topk_select_kernel(TopkState* st, uint32_t* ghist, int shift) {
    const int64_t t = blockIdx.x;
    __shared__ uint64_t sc[2][256];
    const TopkState s0 = st[t];  // read by every thread before any write
    const uint32_t hv = ghist[t * 256 + (255 - threadIdx.x)];
    ghist[t * 256 + (255 - threadIdx.x)] = 0u;
    int sel;
    int64_t cum;
    if (topk_digit_choice(hv, s0.remaining, sc, &sel, &cum)) {
        st[t].prefix = (uint64_t)((K)s0.prefix | ((K)sel << shift));
        st[t].pmask = (uint64_t)((K)s0.pmask | ((K)255 << shift));
        st[t].remaining = s0.remaining - cum;
    }
}

// per chunk: keys above and equal to the threshold (the final prefix)
template <typename T>
__global__ __launch_bounds__(kTopkChunkThreads) void gtt_topk_count_kernel(const T* __restrict__ coef, int64_t N,
                                                                           int64_t nch, const TopkState* __restrict__ st,
                                                                           uint32_t* __restrict__ cnt) {
    using K = typename TopkKey<T>::K;
    __shared__ uint32_t red[2];
    const int64_t t = blockIdx.y;
    const int64_t c0 = (int64_t)blockIdx.x * kTopkChunk;
    const int64_t c1 = c0 + kTopkChunk < N ? c0 + kTopkChunk : N;
    if (threadIdx.x < 2) red[threadIdx.x] = 0u;
    __syncthreads();
    const K thr = (K)st[t].prefix;
    const T* c = coef + t * N;
    uint32_t gt = 0, eq = 0;
    for (int64_t i = c0 + threadIdx.x; i < c1; i += kTopkChunkThreads) {
        const K key = topk_key(c[i]);
        gt += key > thr;
        eq += key == thr;
    }
    if (gt) atomicAdd(&red[0], gt);
    if (eq) atomicAdd(&red[1], eq);
    __syncthreads();
    if (threadIdx.x < 2) cnt[(t * nch + blockIdx.x) * 2 + threadIdx.x] = red[threadIdx.x];
}

// per instance: each chunk's output offset and the equal keys before it
__global__ __launch_bounds__(256) void gtt_topk_scan_kernel(const TopkState* __restrict__ st,
                                                            const uint32_t* __restrict__ cnt,
                                                            int64_t* __restrict__ off, int64_t nch) {
    __shared__ int64_t sg[256], se[256];
    const int64_t t = blockIdx.x;
    const int64_t per = (nch + 255) / 256;
    const int64_t a = (int64_t)threadIdx.x * per;
    const int64_t b = a + per < nch ? a + per : nch;
    const uint32_t* ct = cnt + t * nch * 2;
    int64_t g = 0, e = 0;
    for (int64_t c = a; c < b; ++c) {
        g += ct[2 * c];
        e += ct[2 * c + 1];
    }
    // exclusive scan of the 256 ranges, in order: an inclusive scan over the
    // threads, then each range's own counts taken off
    const int64_t g0 = g, e0 = e;
    for (int o = 1; o < 256; o <<= 1) {
        sg[threadIdx.x] = g;
        se[threadIdx.x] = e;
        __syncthreads();
        if ((int)threadIdx.x >= o) {
            g += sg[threadIdx.x - o];
            e += se[threadIdx.x - o];
        }
        __syncthreads();
    }
    const int64_t need_eq = st[t].remaining;
    g -= g0;
    e -= e0;
    int64_t* ot = off + t * nch * 2;
    for (int64_t c = a; c < b; ++c) {
        ot[2 * c] = g + (e < need_eq ? e : need_eq);  // output position of the chunk's first element
        ot[2 * c + 1] = e;                            // equal keys before the chunk
        g += ct[2 * c];
        e += ct[2 * c + 1];
    }
}

// per chunk: its elements above the threshold and the equal ones still
// needed, in index order, at the chunk's output offset; with rec, also the
// chunk of the dense sparse vector (kept values, zeros elsewhere), which
// replaces a zero fill and a scatter (a chunk reads and writes only its own
// elements, so rec may be coef)
template <typename T>
__global__ __launch_bounds__(kTopkChunkThreads) void gtt_topk_write_kernel(
    const T* coef, int64_t N, int64_t nch, const TopkState* __restrict__ st, const int64_t* __restrict__ off,
    int64_t k, int64_t* __restrict__ idx, T* __restrict__ val, T* rec) {
    using K = typename TopkKey<T>::K;
    __shared__ uint32_t wsum[kTopkChunkThreads / 64];
    const int64_t t = blockIdx.y;
    const int64_t c0 = (int64_t)blockIdx.x * kTopkChunk;
    const int64_t c1 = c0 + kTopkChunk < N ? c0 + kTopkChunk : N;
    const K thr = (K)st[t].prefix;
    const int64_t need_eq = st[t].remaining;
    const T* c = coef + t * N;
    int64_t out = off[(t * nch + blockIdx.x) * 2];
    int64_t eq_seen = off[(t * nch + blockIdx.x) * 2 + 1];
    int64_t* oi = idx + t * k;
    T* ov = val + t * k;
    for (int64_t base = c0; base < c1; base += kTopkChunkThreads) {  // uniform loop
        const int64_t i = base + threadIdx.x;
        const bool in = i < c1;
        const T v = in ? c[i] : from_c<T>(czero<typename Tr<T>::C>());
        const K key = in ? topk_key(v) : (K)0;
        const bool gt = in && key > thr;
        const bool eq = in && key == thr;
        uint32_t eq_tot;
        const uint32_t eq_rank = block_excl_count<kTopkChunkThreads>(eq, wsum, &eq_tot);
        const bool take = gt || (eq && eq_seen + (int64_t)eq_rank < need_eq);
        uint32_t take_tot;
        const uint32_t pos = block_excl_count<kTopkChunkThreads>(take, wsum, &take_tot);
        if (take) {
            oi[out + pos] = i;
            ov[out + pos] = v;
        }
        if (rec && in) rec[t * N + i] = take ? v : from_c<T>(czero<typename Tr<T>::C>());
        eq_seen += eq_tot;
        out += take_tot;
    }
}

// chunked form: few instances, large N
__host__ __device__ inline bool topk_chunked(int64_t N, int64_t batch) {
    return batch < 512 && N >= 4 * (int64_t)kTopkChunk;
}
// workspace bytes of the chunked form (0 otherwise), in 256-byte sections
__host__ __device__ inline size_t topk_ws_bytes(int64_t N, int64_t batch) {
    if (!topk_chunked(N, batch)) return 0;
    const int64_t nch = (N + kTopkChunk - 1) / kTopkChunk;
    auto r = [](size_t x) { return (x + 255) & ~(size_t)255; };
    return r((size_t)batch * sizeof(TopkState)) + r((size_t)batch * 256 * 4) + r((size_t)(batch * nch) * 8) +
           r((size_t)(batch * nch) * 16);
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
