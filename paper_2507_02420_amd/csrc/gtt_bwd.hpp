// Backward of one digit group (the paper has no derivatives; the convention
// is stated in gtt.h).  For a loss L and y = G x, with the digit passes of a
// group applied in digit order, the gradient w.r.t. W collects, for every
// digit s of the group and every fibre of digit s, the outer product c a^H of
// the cotangent c at the output of the pass on digit s and the activation a at
// its input; the gradient at the group's input is W^H applied along every
// digit of the group to the cotangent at its output.
//
// One work-group owns one tile (same geometry as the forward pass of this
// group).  It holds three tiles in LDS: the group input a_in (A), a
// recomputation buffer (Tt) and the cotangent (Ct).  For s = k-1 down to 0 it
// recomputes the input of the pass on digit s from A, accumulates the
// per-fibre outer products into a work-group accumulator of b*b values, and
// applies W^H along digit s to Ct.  Finally Ct (the cotangent at the group's
// input) is written out and the accumulator goes to this work-group's slot of
// the partial-sum buffer.  All sums run in a fixed order (deterministic).
#pragma once

#include "gtt_args.hpp"
#include "gtt_pass.hpp"
#include "gtt_types.hpp"

namespace gtt {

struct BwdArgs {
    PassArgs p;          // tile geometry; p.in = a_in, p.out = c_in, p.W = W
    const void* c_out;   // cotangent at the group's output (storage dtype)
    void* partials;      // [gridDim.x][b*b], compute dtype
    int32_t b;
};

// W (or W^H when adj) along digit j of every fibre of the tile, in place.
// Runtime radix b <= MAXB; a thread owns whole fibres, held in registers.
template <typename C, int MAXB>
__device__ __forceinline__ void digit_apply(C* tile, const C* Wl, const PassArgs& a, int b, int j,
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
            if (q < b) v[q] = tile[lds_phys(lam0 + q * step, a.pad_shift)];
        C o[MAXB];
#pragma unroll
        for (int r = 0; r < MAXB; ++r) {
            if (r < b) {
                C acc = czero<C>();
#pragma unroll
                for (int q = 0; q < MAXB; ++q)
                    if (q < b) acc = cmac(acc, Wl[r * b + q], v[q]);
                o[r] = acc;
            }
        }
#pragma unroll
        for (int r = 0; r < MAXB; ++r)
            if (r < b) tile[lds_phys(lam0 + r * step, a.pad_shift)] = o[r];
    }
}

// acc[r*b+q] += sum over fibres of digit j of Ct[r] * conj(Tt[q]), fixed order.
template <typename C>
__device__ __forceinline__ void gw_sweep(const C* Ct, const C* Tt, C* red, C* acc, const PassArgs& a, int b,
                                         int j, uint32_t rows) {
    const uint32_t Cm = (1u << a.logC) - 1u;
    const uint32_t F = (rows << a.logC) / (uint32_t)b;
    const uint32_t bj = (uint32_t)a.bpow[j];
    const uint32_t bj1 = (uint32_t)a.bpow[j + 1];
    const uint32_t step = bj << a.logC;
    const int bb = b * b;
    const int tpp = kThreads / bb;  // threads per (r, q) pair
    const int t = threadIdx.x;
    C s = czero<C>();
    if (t < bb * tpp) {
        const int e = t % bb, part = t / bb;
        const int r = e / b, q = e - r * b;
        for (uint32_t f = part; f < F; f += tpp) {
            const uint32_t c = f & Cm;
            const uint32_t f1 = f >> a.logC;
            const uint32_t Q = fdiv(f1, a.divb[j]);
            const uint32_t glo = f1 - Q * bj;
            const uint32_t lam0 = ((Q * bj1 + glo) << a.logC) | c;
            s = cmac_conj(s, Ct[lds_phys(lam0 + r * step, a.pad_shift)], Tt[lds_phys(lam0 + q * step, a.pad_shift)]);
        }
    }
    red[t] = s;
    __syncthreads();
    if (t < bb) {
        C tot = acc[t];
        for (int part = 0; part < tpp; ++part) tot = cadd(tot, red[part * bb + t]);
        acc[t] = tot;
    }
    __syncthreads();
}

template <typename T, int MAXB>
__global__ __launch_bounds__(kThreads) void gtt_bwd_kernel(BwdArgs ba) {
    using C = typename Tr<T>::C;
    const PassArgs& a = ba.p;
    const int b = ba.b;
    const int bb = b * b;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const uint32_t rows = (uint32_t)a.P * (uint32_t)a.G;
    const uint32_t tileE = rows << a.logC;
    const uint32_t tileP = lds_tile_elems(tileE, a.pad_shift);
    C* sW = reinterpret_cast<C*>(smem_raw);
    C* sWH = sW + MAXB * MAXB;
    C* acc = sWH + MAXB * MAXB;
    C* red = acc + MAXB * MAXB;
    C* A = red + kThreads;
    C* Tt = A + tileP;
    C* Ct = Tt + tileP;
    {
        const C* __restrict__ Wg = static_cast<const C*>(a.W);
        for (int e = threadIdx.x; e < bb; e += kThreads) {
            const int r = e / b, q = e - r * b;
            sW[e] = Wg[e];
            sWH[e] = cconj(Wg[q * b + r]);
            acc[e] = czero<C>();
        }
    }
    __syncthreads();
    for (int64_t t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
        tile_load<T, C>(A, a, static_cast<const T*>(a.in), t, rows);
        tile_load<T, C>(Ct, a, static_cast<const T*>(ba.c_out), t, rows);
        __syncthreads();
        for (int s = a.k - 1; s >= 0; --s) {
            // input of the pass on digit s: digits 0..s-1 of the group applied to A
            if (s == 0) {
                gw_sweep<C>(Ct, A, red, acc, a, b, s, rows);
            } else {
                for (uint32_t i = threadIdx.x; i < tileP; i += kThreads) Tt[i] = A[i];
                __syncthreads();
                for (int j = 0; j < s; ++j) {
                    digit_apply<C, MAXB>(Tt, sW, a, b, j, rows);
                    __syncthreads();
                }
                gw_sweep<C>(Ct, Tt, red, acc, a, b, s, rows);
            }
            digit_apply<C, MAXB>(Ct, sWH, a, b, s, rows);
            __syncthreads();
        }
        // out is null for the first digit group when only gW is wanted
        if (a.out) tile_store<T, C>(Ct, a, static_cast<T*>(a.out), t, rows);
        __syncthreads();
    }
    C* part = static_cast<C*>(ba.partials) + (size_t)blockIdx.x * bb;
    for (int e = threadIdx.x; e < bb; e += kThreads) part[e] = acc[e];
}

// Fixed-order sum of partial vectors of bb values: work-group w sums the
// parts of its contiguous range [w*n/G, (w+1)*n/G) (interleaved chains inside
// the range, then the chains in order) into out[w].  Two launches (G blocks,
// then one block over the G results) give a deterministic total.
template <typename C>
__global__ __launch_bounds__(kThreads) void gtt_reduce_kernel(const C* __restrict__ partials, int64_t nparts,
                                                              int bb, C* __restrict__ out) {
    __shared__ C red[kThreads];
    const int t = threadIdx.x;
    const int chains = kThreads / bb;
    const int64_t lo = (int64_t)blockIdx.x * nparts / gridDim.x;
    const int64_t hi = (int64_t)(blockIdx.x + 1) * nparts / gridDim.x;
    C s = czero<C>();
    if (t < chains * bb) {
        const int e = t % bb, ch = t / bb;
        int64_t p = lo + ch;
        for (; p + 3 * chains < hi; p += 4 * chains) {
            const C v0 = partials[p * bb + e];
            const C v1 = partials[(p + chains) * bb + e];
            const C v2 = partials[(p + 2 * chains) * bb + e];
            const C v3 = partials[(p + 3 * chains) * bb + e];
            s = cadd(cadd(s, v0), v1);
            s = cadd(cadd(s, v2), v3);
        }
        for (; p < hi; p += chains) s = cadd(s, partials[p * bb + e]);
    }
    red[t] = s;
    __syncthreads();
    if (t < bb) {
        C tot = czero<C>();
        for (int ch = 0; ch < chains; ++ch) tot = cadd(tot, red[ch * bb + t]);
        out[(size_t)blockIdx.x * bb + t] = tot;
    }
}

}  // namespace gtt
