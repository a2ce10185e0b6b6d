// Backward of one digit group (the paper has no derivatives; the convention
// is stated in gtt.h).  For a loss L and y = G x, with the digit passes of a
// group applied in digit order 0..k-1, the gradient w.r.t. the matrix of
// digit s collects, over the fibres of digit s, the outer products c a^H of
// the cotangent c at the output of the pass on digit s and the activation a
// at its input; the gradient at the group's input is the adjoint of every
// digit pass of the group applied to the cotangent at its output.
//
// One work-group owns one tile (P hi blocks x G group positions x C lo
// columns, as in the forward pass).  Its LDS holds `nslots` tiles: slot 0 is
// the group input a_0, slot 1 the cotangent, slots 2.. hold activations
// a_s.  The digits are reversed from k-1 down to 0; the cotangent moves down
// one digit at a time (adjoint pass), while the activation a_s that digit s
// needs is rebuilt from a held one by forward passes.  How many forward
// passes that takes depends on how many slots fit: the host computes an
// optimal checkpoint schedule for the slot count (with k+1 slots every
// activation is computed once: k-1 forward passes, k gradient sweeps, k
// adjoint passes) and the kernel executes it as a list of operations.
//
// The gradient is accumulated in FP64 (complex FP64 for complex data) for
// every storage type: per thread over the fibres of a tile, per work-group
// over its tiles, and in the fixed-order reduction of the work-groups'
// partial vectors; it is rounded to the compute dtype once, at the end.
// All sums run in a fixed order (deterministic).
#pragma once

#include "gtt_args.hpp"
#include "gtt_pass.hpp"
#include "gtt_types.hpp"

namespace gtt {

// schedule operations (uint16): bits 0-1 kind, 2-7 digit, 8-11 src, 12-15 dst
enum BwdOpKind : int { kOpFwd = 0, kOpGw = 1, kOpAdj = 2 };
__host__ __device__ constexpr uint16_t bwd_op(int kind, int digit, int src, int dst) {
    return (uint16_t)(kind | (digit << 2) | (src << 8) | (dst << 12));
}

struct BwdArgs {
    PassArgs p;          // tile geometry; p.in = a_in, p.out = c_in, p.W = W table
    const void* c_out;   // cotangent at the group's output (storage dtype)
    void* partials;      // [gridDim.x][wslot], accumulation dtype
    int32_t nops;
    int32_t nslots;      // LDS tiles (>= 3)
    int32_t wloc;        // entries of the staged matrices and of the accumulator
    int32_t wslot;       // entries of one partial vector (the W table's layout)
    int32_t nf;          // matrices staged: factor i is f_b[i] x f_b[i], at
                         // f_goff[i] in the W table and f_loff[i] in LDS
    int32_t f_goff[kMaxDigits];
    int32_t f_b[kMaxDigits];
    int32_t f_loff[kMaxDigits];
    int32_t lofs[kMaxDigits];  // LDS offset of the matrix of group digit j
    uint16_t ops[kMaxBwdOps];
};

// accumulation type of the weight gradient
template <typename C>
struct AccOf {
    using type = C;
};
template <>
struct AccOf<float> {
    using type = double;
};
template <>
struct AccOf<cf> {
    using type = cd;
};

__device__ __forceinline__ double acc_zero(double) { return 0.0; }
__device__ __forceinline__ cd acc_zero(cd) { return cd{0.0, 0.0}; }
__device__ __forceinline__ double acc_add(double a, double b) { return a + b; }
__device__ __forceinline__ cd acc_add(cd a, cd b) { return cd{a.re + b.re, a.im + b.im}; }

// s + c * conj(a), products and sums in FP64 (a product of two floats is
// exact in FP64)
__device__ __forceinline__ double acc_mac_conj(double s, float c, float a) {
    return __builtin_fma((double)c, (double)a, s);
}
__device__ __forceinline__ double acc_mac_conj(double s, double c, double a) { return __builtin_fma(c, a, s); }
__device__ __forceinline__ cd acc_mac_conj(cd s, cf c, cf a) {
    const double cr = c.re, ci = c.im, ar = a.re, ai = a.im;
    s.re = __builtin_fma(cr, ar, s.re);
    s.re = __builtin_fma(ci, ai, s.re);
    s.im = __builtin_fma(ci, ar, s.im);
    s.im = __builtin_fma(-cr, ai, s.im);
    return s;
}
__device__ __forceinline__ cd acc_mac_conj(cd s, cd c, cd a) { return cmac_conj(s, c, a); }

// accumulator -> compute dtype (one rounding for float / complex float)
__device__ __forceinline__ float acc_to(double v, float*) { return (float)v; }
__device__ __forceinline__ double acc_to(double v, double*) { return v; }
__device__ __forceinline__ cf acc_to(cd v, cf*) { return cf{(float)v.re, (float)v.im}; }
__device__ __forceinline__ cd acc_to(cd v, cd*) { return v; }

// dst = (W or W^H along digit j) src, runtime radix b <= MAXB; a thread owns
// whole fibres: it reads all b values of a fibre into registers before it
// writes any, so dst may equal src.
template <typename C, int MAXB>
__device__ __forceinline__ void digit_apply(const C* src, C* dst, const C* Wl, const PassArgs& a, int b, int j,
                                            uint32_t rows) {
    const uint32_t Cm = (1u << a.logC) - 1u;
    const uint32_t F = (rows << a.logC) / (uint32_t)b;
    const uint32_t bj = (uint32_t)a.bpow[j];
    const uint32_t bj1 = (uint32_t)a.bpow[j + 1];
    const uint32_t step = bj << a.logC;
    for (uint32_t f = threadIdx.x; f < F; f += kThreads) {
        const uint32_t c = f & Cm;
        const uint32_t f1 = f >> a.logC;
        const uint32_t Q = fdiv(f1, a.divb[j]);
        const uint32_t glo = f1 - Q * bj;
        const uint32_t lam0 = ((Q * bj1 + glo) << a.logC) | c;
        C v[MAXB];
#pragma unroll
        for (int q = 0; q < MAXB; ++q)
            if (q < b) v[q] = src[lds_phys(lam0 + q * step, a.pad_shift)];
#pragma unroll
        for (int r = 0; r < MAXB; ++r) {
            if (r < b) {
                C acc = czero<C>();
#pragma unroll
                for (int q = 0; q < MAXB; ++q)
                    if (q < b) acc = cmac(acc, Wl[r * b + q], v[q]);
                dst[lds_phys(lam0 + r * step, a.pad_shift)] = acc;
            }
        }
    }
}

// acc[r*b+q] += sum over the fibres of digit j of Ct[r] * conj(Tt[q]), fixed
// order.  b*b <= kThreads: kThreads/(b*b) threads per (r, q) pair, each over
// an interleaved share of the fibres, then folded in order; larger matrices:
// one thread per pair (several pairs a thread), over all fibres in order.
template <typename C, typename Acc>
__device__ __forceinline__ void gw_sweep(const C* Ct, const C* Tt, Acc* red, Acc* acc, const PassArgs& a, int b,
                                         int j, uint32_t rows) {
    const uint32_t Cm = (1u << a.logC) - 1u;
    const uint32_t F = (rows << a.logC) / (uint32_t)b;
    const uint32_t bj = (uint32_t)a.bpow[j];
    const uint32_t bj1 = (uint32_t)a.bpow[j + 1];
    const uint32_t step = bj << a.logC;
    const int bb = b * b;
    const int t = threadIdx.x;
    auto fibre = [&](uint32_t f) {
        const uint32_t c = f & Cm;
        const uint32_t f1 = f >> a.logC;
        const uint32_t Q = fdiv(f1, a.divb[j]);
        const uint32_t glo = f1 - Q * bj;
        return ((Q * bj1 + glo) << a.logC) | c;
    };
    if (bb <= kThreads) {
        const int tpp = kThreads / bb;  // threads per (r, q) pair
        Acc s = acc_zero(Acc{});
        if (t < bb * tpp) {
            const int e = t % bb, part = t / bb;
            const int r = e / b, q = e - r * b;
            for (uint32_t f = part; f < F; f += tpp) {
                const uint32_t lam0 = fibre(f);
                s = acc_mac_conj(s, Ct[lds_phys(lam0 + r * step, a.pad_shift)],
                                 Tt[lds_phys(lam0 + q * step, a.pad_shift)]);
            }
        }
        red[t] = s;
        __syncthreads();
        if (t < bb) {
            Acc tot = acc[t];
            for (int part = 0; part < tpp; ++part) tot = acc_add(tot, red[part * bb + t]);
            acc[t] = tot;
        }
    } else {
        for (int e = t; e < bb; e += kThreads) {
            const int r = e / b, q = e - r * b;
            Acc s = acc[e];
            for (uint32_t f = 0; f < F; ++f) {
                const uint32_t lam0 = fibre(f);
                s = acc_mac_conj(s, Ct[lds_phys(lam0 + r * step, a.pad_shift)],
                                 Tt[lds_phys(lam0 + q * step, a.pad_shift)]);
            }
            acc[e] = s;
        }
    }
    __syncthreads();
}

__host__ __device__ constexpr size_t bwd_align16(size_t v) { return (v + 15) & ~(size_t)15; }

template <typename T, int MAXB>
__global__ __launch_bounds__(kThreads) void gtt_bwd_kernel(BwdArgs ba) {
    using C = typename Tr<T>::C;
    using Acc = typename AccOf<C>::type;
    const PassArgs& a = ba.p;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const uint32_t rows = (uint32_t)a.P * (uint32_t)a.G;
    const uint32_t tileE = rows << a.logC;
    const uint32_t tileP = lds_tile_elems(tileE, a.pad_shift);
    const int wloc = ba.wloc;
    // [acc: wloc][red: kThreads][W: wloc][W^H: wloc][slots: nslots x tileP]
    unsigned char* pb = smem_raw;
    Acc* acc = reinterpret_cast<Acc*>(pb);
    pb += bwd_align16((size_t)wloc * sizeof(Acc));
    Acc* red = reinterpret_cast<Acc*>(pb);
    pb += (size_t)kThreads * sizeof(Acc);
    C* sW = reinterpret_cast<C*>(pb);
    pb += bwd_align16((size_t)wloc * sizeof(C));
    C* sWH = reinterpret_cast<C*>(pb);
    pb += bwd_align16((size_t)wloc * sizeof(C));
    C* slot0 = reinterpret_cast<C*>(pb);
    auto slot = [&](int i) { return slot0 + (size_t)i * tileP; };
    {
        const C* __restrict__ Wg = static_cast<const C*>(a.W);
        for (int i = 0; i < ba.nf; ++i) {
            const int b = ba.f_b[i], bb = b * b;
            const C* Wf = Wg + ba.f_goff[i];
            C* dW = sW + ba.f_loff[i];
            C* dH = sWH + ba.f_loff[i];
            for (int e = threadIdx.x; e < bb; e += kThreads) {
                const int r = e / b, q = e - r * b;
                dW[e] = Wf[e];
                dH[e] = cconj(Wf[q * b + r]);
            }
        }
        for (int e = threadIdx.x; e < wloc; e += kThreads) acc[e] = acc_zero(Acc{});
    }
    __syncthreads();
    C* Ct = slot(1);
    for (int64_t t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
        tile_load<T, C>(slot(0), a, static_cast<const T*>(a.in), t, rows);
        tile_load<T, C>(Ct, a, static_cast<const T*>(ba.c_out), t, rows);
        __syncthreads();
        for (int o = 0; o < ba.nops; ++o) {
            const int op = ba.ops[o];
            const int kind = op & 3, j = (op >> 2) & 63, src = (op >> 8) & 15, dst = (op >> 12) & 15;
            const int b = a.rad[j];
            if (kind == kOpFwd) {
                digit_apply<C, MAXB>(slot(src), slot(dst), sW + ba.lofs[j], a, b, j, rows);
                __syncthreads();
            } else if (kind == kOpGw) {
                gw_sweep<C, Acc>(Ct, slot(src), red, acc + ba.lofs[j], a, b, j, rows);
            } else if (j != 0 || a.out) {
                // (the cotangent at the input of digit 0 is needed only when
                // it is stored: out is null for the first digit group when
                // only gW is wanted)
                digit_apply<C, MAXB>(Ct, Ct, sWH + ba.lofs[j], a, b, j, rows);
                __syncthreads();
            }
        }
        if (a.out) tile_store<T, C>(Ct, a, static_cast<T*>(a.out), t, rows);
        __syncthreads();
    }
    // this work-group's partial vector in the W table's layout (zero outside
    // the matrices of this group's digits)
    Acc* part = static_cast<Acc*>(ba.partials) + (size_t)blockIdx.x * ba.wslot;
    for (int e = threadIdx.x; e < ba.wslot; e += kThreads) {
        Acc v = acc_zero(Acc{});
        for (int i = 0; i < ba.nf; ++i) {
            const int d = e - ba.f_goff[i];
            if (d >= 0 && d < ba.f_b[i] * ba.f_b[i]) v = acc[ba.f_loff[i] + d];
        }
        part[e] = v;
    }
}

// Fixed-order sum of partial vectors of bb accumulation-type values:
// work-group w sums the parts of its contiguous range [w*n/G, (w+1)*n/G)
// (bb <= kThreads: interleaved chains inside the range, then the chains in
// order; larger vectors: one thread per entry over the range in order) into
// out[w], converted to Out.  Two launches (G work-groups into accumulation-
// type vectors, then one over the G results into the compute dtype) give a
// deterministic total.
template <typename Acc, typename Out>
__global__ __launch_bounds__(kThreads) void gtt_reduce_kernel(const Acc* __restrict__ partials, int64_t nparts,
                                                              int bb, Out* __restrict__ out) {
    __shared__ Acc red[kThreads];
    const int t = threadIdx.x;
    const int64_t lo = (int64_t)blockIdx.x * nparts / gridDim.x;
    const int64_t hi = (int64_t)(blockIdx.x + 1) * nparts / gridDim.x;
    if (bb > kThreads) {
        for (int e = t; e < bb; e += kThreads) {
            Acc s = acc_zero(Acc{});
            for (int64_t p = lo; p < hi; ++p) s = acc_add(s, partials[p * bb + e]);
            out[(size_t)blockIdx.x * bb + e] = acc_to(s, (Out*)nullptr);
        }
        return;
    }
    const int chains = kThreads / bb;
    Acc s = acc_zero(Acc{});
    if (t < chains * bb) {
        const int e = t % bb, ch = t / bb;
        int64_t p = lo + ch;
        for (; p + 3 * chains < hi; p += 4 * chains) {
            const Acc v0 = partials[p * bb + e];
            const Acc v1 = partials[(p + chains) * bb + e];
            const Acc v2 = partials[(p + 2 * chains) * bb + e];
            const Acc v3 = partials[(p + 3 * chains) * bb + e];
            s = acc_add(acc_add(s, v0), v1);
            s = acc_add(acc_add(s, v2), v3);
        }
        for (; p < hi; p += chains) s = acc_add(s, partials[p * bb + e]);
    }
    red[t] = s;
    __syncthreads();
    if (t < bb) {
        Acc tot = acc_zero(Acc{});
        for (int ch = 0; ch < chains; ++ch) tot = acc_add(tot, red[ch * bb + t]);
        out[(size_t)blockIdx.x * bb + t] = acc_to(tot, (Out*)nullptr);
    }
}

// Per-storage-type launchers of the backward and of the gW reduction; each
// bwd_<dtype>.hip translation unit instantiates them for one storage type.
template <typename T>
hipError_t launch_bwd_t(const BwdArgs& a, int maxb, unsigned grid, size_t lds, hipStream_t s) {
    const void* k = maxb <= 8    ? reinterpret_cast<const void*>(gtt_bwd_kernel<T, 8>)
                    : maxb <= 16 ? reinterpret_cast<const void*>(gtt_bwd_kernel<T, 16>)
                                 : reinterpret_cast<const void*>(gtt_bwd_kernel<T, 32>);
    if (maxb > 32) return hipErrorInvalidValue;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    if (maxb <= 8)
        hipLaunchKernelGGL((gtt_bwd_kernel<T, 8>), dim3(grid), dim3(kThreads), lds, s, a);
    else if (maxb <= 16)
        hipLaunchKernelGGL((gtt_bwd_kernel<T, 16>), dim3(grid), dim3(kThreads), lds, s, a);
    else
        hipLaunchKernelGGL((gtt_bwd_kernel<T, 32>), dim3(grid), dim3(kThreads), lds, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_reduce_t(const void* partials, int64_t nparts, int bb, void* out, hipStream_t s) {
    using C = typename Tr<T>::C;
    using Acc = typename AccOf<C>::type;
    Acc* mid = const_cast<Acc*>(static_cast<const Acc*>(partials)) + (size_t)nparts * bb;
    const int g1 = (int)(nparts < kReduceBlocks ? nparts : kReduceBlocks);
    hipLaunchKernelGGL((gtt_reduce_kernel<Acc, Acc>), dim3(g1), dim3(kThreads), 0, s,
                       static_cast<const Acc*>(partials), nparts, bb, mid);
    hipLaunchKernelGGL((gtt_reduce_kernel<Acc, C>), dim3(1), dim3(kThreads), 0, s, (const Acc*)mid, (int64_t)g1,
                       bb, static_cast<C*>(out));
    return hipGetLastError();
}

}  // namespace gtt

// Instantiation of the launchers for one storage type (NAME: the dtype's
// short name used in the launcher symbols, T: the storage type).
#define GTT_BWD_INSTANTIATE(NAME, T)                                                                     \
    namespace gtt {                                                                                      \
    hipError_t launch_bwd_##NAME(const BwdArgs& a, int maxb, unsigned grid, size_t lds, hipStream_t s) { \
        return launch_bwd_t<T>(a, maxb, grid, lds, s);                                                   \
    }                                                                                                    \
    hipError_t launch_reduce_##NAME(const void* partials, int64_t nparts, int bb, void* out,            \
                                    hipStream_t s) {                                                     \
        return launch_reduce_t<T>(partials, nparts, bb, out, s);                                         \
    }                                                                                                    \
    }
