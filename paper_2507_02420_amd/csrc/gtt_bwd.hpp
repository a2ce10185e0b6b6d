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

#include <map>
#include <mutex>
#include <tuple>

#include "gtt_args.hpp"
#include "gtt_mfma.hpp"
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

// dst = (W or W^H along digit j) src, radix B compiled in; a thread owns
// whole fibres: it reads all B values of a fibre into registers before it
// writes any, so dst may equal src.  LIN: an unpadded tile (linear LDS
// positions).
template <typename C, int B, bool LIN>
__device__ __forceinline__ void digit_apply_b(const C* src, C* dst, const C* Wl, const PassArgs& a, int j,
                                              uint32_t rows) {
    const uint32_t Cm = (1u << a.logC) - 1u;
    const uint32_t F = (rows << a.logC) / (uint32_t)B;
    const uint32_t bj = (uint32_t)a.bpow[j];
    const uint32_t bj1 = (uint32_t)a.bpow[j + 1];
    const uint32_t step = bj << a.logC;
    auto phys = [&](uint32_t x) { return LIN ? x : lds_phys(x, a.pad_shift); };
    for (uint32_t f = threadIdx.x; f < F; f += kThreads) {
        const uint32_t c = f & Cm;
        const uint32_t f1 = f >> a.logC;
        const uint32_t Q = fdiv(f1, a.divb[j]);
        const uint32_t glo = f1 - Q * bj;
        const uint32_t lam0 = ((Q * bj1 + glo) << a.logC) | c;
        C v[B];
#pragma unroll
        for (int q = 0; q < B; ++q) v[q] = src[phys(lam0 + (uint32_t)q * step)];
#pragma unroll
        for (int r = 0; r < B; ++r) {
            C acc = cmul(Wl[r * B], v[0]);
#pragma unroll
            for (int q = 1; q < B; ++q) acc = cmac(acc, Wl[r * B + q], v[q]);
            dst[phys(lam0 + (uint32_t)r * step)] = acc;
        }
    }
}

#define GTT_DA_CASE(B)                                                   \
    case B:                                                              \
        if constexpr (B <= LIM) digit_apply_b<C, B, LIN>(src, dst, Wl, a, j, rows); \
        break;
template <typename C, bool LIN, int LIM>
__device__ __forceinline__ void digit_apply_sw(const C* src, C* dst, const C* Wl, const PassArgs& a, int b, int j,
                                               uint32_t rows) {
    switch (b) {
        GTT_DA_CASE(2) GTT_DA_CASE(3) GTT_DA_CASE(4) GTT_DA_CASE(5) GTT_DA_CASE(6) GTT_DA_CASE(7)
        GTT_DA_CASE(8) GTT_DA_CASE(9) GTT_DA_CASE(10) GTT_DA_CASE(11) GTT_DA_CASE(12) GTT_DA_CASE(13)
        GTT_DA_CASE(14) GTT_DA_CASE(15) GTT_DA_CASE(16)
        default: break;
    }
}
#undef GTT_DA_CASE

// the same for a runtime radix b <= MAXB: radices up to 8 take the
// compiled-in form, larger ones a loop over b with run-time bounds (compiled
// in, their matrices would be held in registers across the fibre loop and
// spill)
template <typename C, int MAXB>
__device__ __forceinline__ void digit_apply(const C* src, C* dst, const C* Wl, const PassArgs& a, int b, int j,
                                            uint32_t rows) {
    constexpr int LIM = MAXB < 8 ? MAXB : 8;
    if (b <= LIM) {
        if (a.pad_shift == kPadNone) digit_apply_sw<C, true, LIM>(src, dst, Wl, a, b, j, rows);
        else digit_apply_sw<C, false, LIM>(src, dst, Wl, a, b, j, rows);
        return;
    }
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

__device__ __forceinline__ double acc_shfl_down(double v, int d) { return __shfl_down(v, d, 64); }
__device__ __forceinline__ cd acc_shfl_down(cd v, int d) {
    return cd{__shfl_down(v.re, d, 64), __shfl_down(v.im, d, 64)};
}

// The same sums for b <= 8 (4 b*b <= kThreads), a row of the gradient per
// lane: a wave's lanes are (sub, r) pairs, r = lane % b, sub = lane / b
// (64 / b of them), and lane (sub, r) of wave w takes fibres
// f = w * subs + sub + i * 4 * subs: it reads Ct[r] once and Tt[0..b-1] of
// each and keeps the b sums of row r in registers.  The sums are folded over
// sub inside the wave by shuffles (a fixed tree), then the four waves' rows
// are added in wave order into acc.
template <typename C, typename Acc, int B, bool LIN>
__device__ __forceinline__ void gw_rows(const C* Ct, const C* Tt, Acc* red, Acc* acc, const PassArgs& a, int j,
                                        uint32_t rows) {
    constexpr int MB = B;
    constexpr int b = B;
    const uint32_t Cm = (1u << a.logC) - 1u;
    const uint32_t F = (rows << a.logC) / (uint32_t)b;
    const uint32_t bj = (uint32_t)a.bpow[j];
    const uint32_t bj1 = (uint32_t)a.bpow[j + 1];
    const uint32_t step = bj << a.logC;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int subs = 64 / b;
    const int sub = lane / b, r = lane - sub * b;
    auto phys = [&](uint32_t x) { return LIN ? x : lds_phys(x, a.pad_shift); };
    Acc s[MB];
#pragma unroll
    for (int q = 0; q < MB; ++q) s[q] = acc_zero(Acc{});
    if (sub < subs) {
        for (uint32_t f = (uint32_t)(wave * subs + sub); f < F; f += (uint32_t)(4 * subs)) {
            const uint32_t c = f & Cm;
            const uint32_t f1 = f >> a.logC;
            const uint32_t Q = fdiv(f1, a.divb[j]);
            const uint32_t glo = f1 - Q * bj;
            const uint32_t lam0 = ((Q * bj1 + glo) << a.logC) | c;
            const C cr = Ct[phys(lam0 + (uint32_t)r * step)];
#pragma unroll
            for (int q = 0; q < MB; ++q) s[q] = acc_mac_conj(s[q], cr, Tt[phys(lam0 + (uint32_t)q * step)]);
        }
    }
    for (int h = 1; h < subs; h <<= 1) {
        const bool take = (sub & (2 * h - 1)) == 0 && sub + h < subs;
#pragma unroll
        for (int q = 0; q < MB; ++q) {
            const Acc o = acc_shfl_down(s[q], h * b);
            if (take) s[q] = acc_add(s[q], o);
        }
    }
    const int bb = b * b;
    if (sub == 0) {
#pragma unroll
        for (int q = 0; q < MB; ++q) red[wave * bb + r * b + q] = s[q];
    }
    __syncthreads();
    const int t = threadIdx.x;
    if (t < bb) {
        Acc tot = acc[t];
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) tot = acc_add(tot, red[w * bb + t]);
        acc[t] = tot;
    }
    __syncthreads();
}

// The row-wise sums for a radix b in 9..16 given at run time, one body for
// all of them (compiled per radix, several bodies in one kernel pushed it
// into scratch): columns q0 .. q0 + qn - 1 (qn <= 8) of each lane's row, the
// waves' rows added into acc one after another in wave order.  The caller
// covers a row in two calls (two passes over the fibres: columns 0..7 and
// 8..b-1, measured faster than an even split).
template <typename C, typename Acc, bool LIN>
__device__ __forceinline__ void gw_rows_rt(const C* Ct, const C* Tt, Acc* acc, const PassArgs& a, int b, int q0,
                                           int qn, int j, uint32_t rows) {
    constexpr int MB = 8;
    const uint32_t Cm = (1u << a.logC) - 1u;
    const uint32_t F = (rows << a.logC) / (uint32_t)b;
    const uint32_t bj = (uint32_t)a.bpow[j];
    const uint32_t bj1 = (uint32_t)a.bpow[j + 1];
    const uint32_t step = bj << a.logC;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int subs = 64 / b;
    const int sub = lane / b, r = lane - sub * b;
    auto phys = [&](uint32_t x) { return LIN ? x : lds_phys(x, a.pad_shift); };
    Acc s[MB];
#pragma unroll
    for (int q = 0; q < MB; ++q) s[q] = acc_zero(Acc{});
    if (sub < subs) {
        for (uint32_t f = (uint32_t)(wave * subs + sub); f < F; f += (uint32_t)(4 * subs)) {
            const uint32_t c = f & Cm;
            const uint32_t f1 = f >> a.logC;
            const uint32_t Q = fdiv(f1, a.divb[j]);
            const uint32_t glo = f1 - Q * bj;
            const uint32_t lam0 = ((Q * bj1 + glo) << a.logC) | c;
            const C cr = Ct[phys(lam0 + (uint32_t)r * step)];
#pragma unroll
            for (int q = 0; q < MB; ++q)
                if (q < qn) s[q] = acc_mac_conj(s[q], cr, Tt[phys(lam0 + (uint32_t)(q0 + q) * step)]);
        }
    }
    for (int h = 1; h < subs; h <<= 1) {
        const bool take = (sub & (2 * h - 1)) == 0 && sub + h < subs;
#pragma unroll
        for (int q = 0; q < MB; ++q) {
            if (q < qn) {
                const Acc o = acc_shfl_down(s[q], h * b);
                if (take) s[q] = acc_add(s[q], o);
            }
        }
    }
    for (int w = 0; w < kThreads / 64; ++w) {
        if (wave == w && sub == 0) {
#pragma unroll
            for (int q = 0; q < MB; ++q)
                if (q < qn) acc[r * b + q0 + q] = acc_add(acc[r * b + q0 + q], s[q]);
        }
        __syncthreads();
    }
}

template <typename C, typename Acc, bool LIN>
__device__ __forceinline__ void gw_rows_sw(const C* Ct, const C* Tt, Acc* red, Acc* acc, const PassArgs& a, int b,
                                           int j, uint32_t rows) {
    switch (b) {
        case 2: gw_rows<C, Acc, 2, LIN>(Ct, Tt, red, acc, a, j, rows); break;
        case 3: gw_rows<C, Acc, 3, LIN>(Ct, Tt, red, acc, a, j, rows); break;
        case 4: gw_rows<C, Acc, 4, LIN>(Ct, Tt, red, acc, a, j, rows); break;
        case 5: gw_rows<C, Acc, 5, LIN>(Ct, Tt, red, acc, a, j, rows); break;
        case 6: gw_rows<C, Acc, 6, LIN>(Ct, Tt, red, acc, a, j, rows); break;
        case 7: gw_rows<C, Acc, 7, LIN>(Ct, Tt, red, acc, a, j, rows); break;
        case 8: gw_rows<C, Acc, 8, LIN>(Ct, Tt, red, acc, a, j, rows); break;
        default: break;
    }
}

__host__ __device__ constexpr size_t bwd_align16(size_t v) { return (v + 15) & ~(size_t)15; }

// W4: the form compiled for four waves per SIMD (at most 128 VGPRs); the
// launch takes it where it fits more work-groups than the unconstrained one
template <bool W4>
struct BwdMinWaves {
    static constexpr int value = W4 ? 4 : 1;
};

template <typename T, int MAXB, bool W4 = false>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(BwdMinWaves<W4>::value))) void gtt_bwd_kernel(
    BwdArgs ba) {
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
    // radices from which the run-time row sums beat the pair sweep (complex
    // data: measured slower at 9 and 11, faster at 16)
    constexpr int kRowsRtMin = (std::is_same<C, cf>::value || std::is_same<C, cd>::value) ? 12 : 9;
    for (int64_t t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
        // run-time radices: element-wise tiles take the scalar address walk
        tile_load<T, C, kThreads, true>(slot(0), a, static_cast<const T*>(a.in), t, rows);
        tile_load<T, C, kThreads, true>(Ct, a, static_cast<const T*>(ba.c_out), t, rows);
        __syncthreads();
        for (int o = 0; o < ba.nops; ++o) {
            const int op = ba.ops[o];
            const int kind = op & 3, j = (op >> 2) & 63, src = (op >> 8) & 15, dst = (op >> 12) & 15;
            const int b = a.rad[j];
            if (kind == kOpFwd) {
                digit_apply<C, MAXB>(slot(src), slot(dst), sW + ba.lofs[j], a, b, j, rows);
                __syncthreads();
            } else if (kind == kOpGw) {
                if (b <= 8 && a.pad_shift == kPadNone)
                    gw_rows_sw<C, Acc, true>(Ct, slot(src), red, acc + ba.lofs[j], a, b, j, rows);
                else if (b <= 8)
                    gw_rows_sw<C, Acc, false>(Ct, slot(src), red, acc + ba.lofs[j], a, b, j, rows);
                else if (MAXB > 8 && b <= 16 && b >= kRowsRtMin && a.pad_shift == kPadNone) {
                    if constexpr (MAXB > 8) {
                        // two passes over the fibres: columns 0..7, then 8..b-1
                        gw_rows_rt<C, Acc, true>(Ct, slot(src), acc + ba.lofs[j], a, b, 0, 8, j, rows);
                        gw_rows_rt<C, Acc, true>(Ct, slot(src), acc + ba.lofs[j], a, b, 8, b - 8, j, rows);
                    }
                } else
                    gw_sweep<C, Acc>(Ct, slot(src), red, acc + ba.lofs[j], a, b, j, rows);
            } else if (j != 0 || a.out) {
                // (the cotangent at the input of digit 0 is needed only when
                // it is stored: out is null for the first digit group when
                // only gW is wanted)
                digit_apply<C, MAXB>(Ct, Ct, sWH + ba.lofs[j], a, b, j, rows);
                __syncthreads();
            }
        }
        if (a.out) tile_store<T, C, false, kThreads, true>(Ct, a, static_cast<T*>(a.out), t, rows);
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

// ---------------------------------------------------------------------------
// Matrix-core backward for radix 16 and 32 (one W for every digit; bf16,
// f16 or float storage): the same per-tile schedule as gtt_bwd_kernel on
// FP32 tiles in LDS, every digit operation a dense contraction on the FP32
// MFMA (16x16x4): forward passes rebuilding activations with W, the gradient
// sums c a^T over the fibres of a digit (four fibres per MFMA, each tile's
// chain added into FP64), and the adjoint passes with W^T.  The waves' FP64
// sums are added in wave order at the end.
// ---------------------------------------------------------------------------
template <typename T>
constexpr bool bwd_mfma_ok() {
    return sizeof(T) == 2 || std::is_same<T, float>::value;
}

template <typename T, int B>
__global__ __launch_bounds__(kThreads) void gtt_bwd_mfma_kernel(BwdArgs ba) {
    static_assert(B == 16 || B == 32, "matrix-core radices");
    static_assert(bwd_mfma_ok<T>(), "real storage with float compute");
    constexpr int NB = B / 16;
    const PassArgs& a = ba.p;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const uint32_t rows = (uint32_t)a.P * (uint32_t)a.G;
    const uint32_t tileE = rows << a.logC;
    const uint32_t tileP = lds_tile_elems(tileE, a.pad_shift);
    // the layout of gtt_bwd_kernel ([acc][red][W][W^H][slots]): the FP64 area
    // acc (B * B values) takes the work-group's sum; W stays in registers
    double* acc = reinterpret_cast<double*>(smem_raw);
    unsigned char* pb = smem_raw;
    pb += bwd_align16((size_t)ba.wloc * sizeof(double));
    pb += (size_t)kThreads * sizeof(double);
    pb += 2 * bwd_align16((size_t)ba.wloc * sizeof(float));
    float* slot0 = reinterpret_cast<float*>(pb);
    auto slot = [&](int i) { return slot0 + (size_t)i * tileP; };
    WFrag<float, B> wf, wt;
    {
        PassArgs aw = a;
        aw.adjoint = 0;
        load_w_frag<float, B>(wf, aw);
        aw.adjoint = 1;  // W^T (real)
        load_w_frag<float, B>(wt, aw);
    }
    double Md[NB][NB][4];
#pragma unroll
    for (int bi = 0; bi < NB; ++bi)
#pragma unroll
        for (int bj = 0; bj < NB; ++bj)
#pragma unroll
            for (int v = 0; v < 4; ++v) Md[bi][bj][v] = 0.0;
    float* Ct = slot(1);
    for (int64_t t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
        tile_load<T, float>(slot(0), a, static_cast<const T*>(a.in), t, rows);
        tile_load<T, float>(Ct, a, static_cast<const T*>(ba.c_out), t, rows);
        __syncthreads();
        for (int o = 0; o < ba.nops; ++o) {
            const int op = ba.ops[o];
            const int kind = op & 3, j = (op >> 2) & 63, src = (op >> 8) & 15, dst = (op >> 12) & 15;
            if (kind == kOpFwd) {
                mfma_pass_f32<B>(slot(src), slot(dst), a, j, rows, wf);
            } else if (kind == kOpGw) {
                mfma_gw_f32<B>(Ct, slot(src), a, j, rows, Md);
            } else if (j != 0 || a.out) {
                // (the cotangent at the input of digit 0 only when it is
                // stored, as in gtt_bwd_kernel)
                mfma_pass_f32<B>(Ct, Ct, a, j, rows, wt);
            }
            __syncthreads();
        }
        if (a.out) tile_store<T, float>(Ct, a, static_cast<T*>(a.out), t, rows);
        __syncthreads();
    }
    // work-group sum in wave order, then this work-group's partial vector
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int w = 0; w < kThreads / 64; ++w) {
        if (wave == w) {
#pragma unroll
            for (int bi = 0; bi < NB; ++bi)
#pragma unroll
                for (int bj = 0; bj < NB; ++bj)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int e = (16 * bi + 4 * (lane >> 4) + v) * B + 16 * bj + (lane & 15);
                        acc[e] = (w == 0 ? 0.0 : acc[e]) + Md[bi][bj][v];
                    }
        }
        __syncthreads();
    }
    double* part = static_cast<double*>(ba.partials) + (size_t)blockIdx.x * ba.wslot;
    for (int e = threadIdx.x; e < ba.wslot; e += kThreads) part[e] = e < B * B ? acc[e] : 0.0;
}

// ---------------------------------------------------------------------------
// Radix-specialised backward on register blocks (one W shared by every
// digit, radix B = 2..5 known at compile time).  The digits of the group are
// taken RD at a time ("blocks"); the host's checkpoint schedule runs over the
// blocks (operation digit field = block index), so an LDS slot holds the
// activation at the start of a block.  A thread owns one B^r-element block of
// the tile (r <= RD digits, the positions of one value of every other digit)
// in registers:
//   - forward over a block: load, apply W along its r digits in registers,
//     store (one LDS round trip for r digits);
//   - gradient and adjoint over a block: load the block's activation and its
//     cotangent, rebuild the r activations inside the block in registers,
//     then for the block's digits from the last down: add the outer products
//     of the digit's fibres into the thread's FP64 accumulators and apply
//     W^H along the digit to the cotangent in registers; store the cotangent
//     (again one LDS round trip for r digits).
// W lives in registers (the adjoint passes read it transposed and
// conjugated); the accumulators too, for the whole launch
// (every block a thread owns, tile after tile, in order), and are summed
// over the work-group once at the end: over the lanes of a wave by a fixed
// shuffle tree, then over the waves in order.
// ---------------------------------------------------------------------------
// digits per register block for storage type T (compute type C) and radix
// b; 0: no radix-specialised kernel
template <typename C>
__host__ __device__ constexpr int bwd_block_digits(int b) {
    if (std::is_same<C, float>::value) return b == 2 ? 4 : (b == 3 || b == 4) ? 2 : b == 5 ? 1 : 0;
    if (std::is_same<C, double>::value) return b == 2 ? 3 : b == 3 ? 2 : (b == 4 || b == 5) ? 1 : 0;
    if (std::is_same<C, cf>::value) return b == 2 ? 3 : (b == 3 || b == 4) ? 1 : 0;
    if (std::is_same<C, cd>::value) return b == 2 ? 2 : (b == 3 || b == 4) ? 1 : 0;
    return 0;
}

// The B^R positions of block f of a group whose first block digit is j:
// lam0 (the block's digits zero) plus m * step, m the block-local index
// (digit j + d at stride B^d).  The padded map lds_phys is additive over
// numbers with disjoint bits; for a power-of-two radix the block positions
// and lam0 have disjoint bits, and an odd radix (3, 5) runs unpadded tiles
// (the map is the identity): phys(lam0 + m * step) = phys(lam0) + phys(m * step).
template <int B, int R>
struct BlockGeom {
    static constexpr int NB = IPow<B, R>::value;
    uint32_t off[NB];
    uint32_t Cm, F, bj, bjr;
    int logC, pad;
    __device__ __forceinline__ BlockGeom(const PassArgs& a, int j, uint32_t rows) {
        Cm = (1u << a.logC) - 1u;
        F = (rows << a.logC) / (uint32_t)NB;
        bj = (uint32_t)a.bpow[j];
        bjr = (uint32_t)a.bpow[j + R];
        logC = a.logC;
        pad = a.pad_shift;
        const uint32_t step = bj << a.logC;
#pragma unroll
        for (int m = 0; m < NB; ++m) off[m] = lds_phys((uint32_t)m * step, pad);
    }
    __device__ __forceinline__ uint32_t base(const PassArgs& a, int j, uint32_t f) const {
        const uint32_t c = f & Cm;
        const uint32_t f1 = f >> logC;
        const uint32_t Q = fdiv(f1, a.divb[j]);
        return lds_phys(((Q * bjr + (f1 - Q * bj)) << logC) | c, pad);
    }
};

// forward over a block: dst = W along digits j..j+R-1 of src (dst may be src);
// NT threads
template <typename C, int B, int R, int NT>
__device__ __forceinline__ void block_fwd(const C* src, C* dst, const C (&w)[B * B], const PassArgs& a, int j,
                                          uint32_t rows) {
    const BlockGeom<B, R> g(a, j, rows);
    constexpr int NB = BlockGeom<B, R>::NB;
    for (uint32_t f = threadIdx.x; f < g.F; f += NT) {
        const uint32_t ph0 = g.base(a, j, f);
        C v[NB];
#pragma unroll
        for (int m = 0; m < NB; ++m) v[m] = src[ph0 + g.off[m]];
        BlockAll<C, B, R, 0>::run(v, w);
#pragma unroll
        for (int m = 0; m < NB; ++m) dst[ph0 + g.off[m]] = v[m];
    }
}

// gradient sums over the fibres of block digit D (cotangent cv, activation av)
template <typename C, typename Acc, int B, int R, int D>
__device__ __forceinline__ void block_gw(const C (&cv)[(IPow<B, R>::value)], const C (&av)[(IPow<B, R>::value)],
                                         Acc (&acc)[B * B]) {
    constexpr int st = IPow<B, D>::value;
    constexpr int NB = IPow<B, R>::value;
#pragma unroll
    for (int base = 0; base < NB; ++base) {
        if ((base / st) % B != 0) continue;  // fibre start: digit D zero
#pragma unroll
        for (int r = 0; r < B; ++r)
#pragma unroll
            for (int q = 0; q < B; ++q)
                acc[r * B + q] = acc_mac_conj(acc[r * B + q], cv[base + r * st], av[base + q * st]);
    }
}

// the block's digits from D down to 0: gradient sums, then the adjoint pass
// (the adjoint of digit 0 only when adj0)
template <typename C, typename Acc, int B, int R, int D>
struct BlockRev {
    __device__ __forceinline__ static void run(C (&cv)[(IPow<B, R>::value)], const C (&acts)[R][(IPow<B, R>::value)],
                                               const C (&w)[B * B], Acc (&acc)[B * B], bool adj0) {
        block_gw<C, Acc, B, R, D>(cv, acts[D], acc);
        if (D > 0 || adj0) block_digit_adj<C, B, R, D>(cv, w);
        BlockRev<C, Acc, B, R, D - 1>::run(cv, acts, w, acc, adj0);
    }
};
template <typename C, typename Acc, int B, int R>
struct BlockRev<C, Acc, B, R, -1> {
    __device__ __forceinline__ static void run(C (&)[(IPow<B, R>::value)], const C (&)[R][(IPow<B, R>::value)],
                                               const C (&)[B * B], Acc (&)[B * B], bool) {}
};

// activations inside the block: acts[d + 1] = W along digit d of acts[d]
template <typename C, int B, int R, int D>
struct BlockActs {
    __device__ __forceinline__ static void run(C (&acts)[R][(IPow<B, R>::value)], const C (&w)[B * B]) {
        if constexpr (D + 1 < R) {
#pragma unroll
            for (int m = 0; m < IPow<B, R>::value; ++m) acts[D + 1][m] = acts[D][m];
            block_digit<C, B, R, D>(acts[D + 1], w);
            BlockActs<C, B, R, D + 1>::run(acts, w);
        }
    }
};

// gradient sums and adjoint over a block; the cotangent is stored back
// unless this is block 0 and the group's input cotangent is not wanted
template <typename C, typename Acc, int B, int R, int NT>
__device__ __forceinline__ void block_gw_adj(C* Ct, const C* act, const C (&w)[B * B], Acc (&acc)[B * B],
                                             const PassArgs& a, int j, uint32_t rows, bool store) {
    const BlockGeom<B, R> g(a, j, rows);
    constexpr int NB = BlockGeom<B, R>::NB;
    for (uint32_t f = threadIdx.x; f < g.F; f += NT) {
        const uint32_t ph0 = g.base(a, j, f);
        C acts[R][NB], cv[NB];
#pragma unroll
        for (int m = 0; m < NB; ++m) {
            acts[0][m] = act[ph0 + g.off[m]];
            cv[m] = Ct[ph0 + g.off[m]];
        }
        BlockActs<C, B, R, 0>::run(acts, w);
        BlockRev<C, Acc, B, R, R - 1>::run(cv, acts, w, acc, store);
        if (store) {
#pragma unroll
            for (int m = 0; m < NB; ++m) Ct[ph0 + g.off[m]] = cv[m];
        }
    }
}

// Complex radix B = 3 or 4, one digit per block: the gradient sums of a
// digit on the FP32 matrix cores, the adjoint on the VALU.  The sum over
// fibres of c a^H is a contraction over the fibre index: with c and a as
// real 8-vectors (B real parts, then B imaginary parts, each part padded with
// zeros to four), one 16x16x4 MFMA
// takes four fibres each of two sets (rows / columns 0-7: set 0, 8-15: set 1;
// lane (m, k) supplies component m % 8 of fibre 4 (m / 8) + k of the set
// group, for the cotangent (A) and the activation (B) alike), and the two
// diagonal 8x8 blocks of D are the set's sums (the off-diagonal blocks
// are not used).  A wave takes its 64 fibres as eight such groups, reading
// the operands from LDS at the fibre positions its lanes computed (a lane
// shuffle) before any lane writes its adjoint back.  Each digit's FP32
// chain over the tile is added into the lane's FP64 sums Md.
template <int B>
__device__ __forceinline__ void block_gw_adj_cmfma(cf* Ct, const cf* act, const cf (&w)[B * B], double (&Md)[4],
                                                   const PassArgs& a, int j, uint32_t rows, bool store, int nt) {
    static_assert(B == 3 || B == 4, "complex radix 3 or 4");
    const BlockGeom<B, 1> g(a, j, rows);
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t m = lane & 15u, kk = lane >> 4;
    const uint32_t comp = (m >> 2) & 1u, r = m & 3u;
    const bool rlive = r < (uint32_t)B;  // radix 3: component rows 3 and 7 are zero padding
    uint32_t offr = g.off[0];
#pragma unroll
    for (int e = 1; e < B; ++e) offr = r == (uint32_t)e ? g.off[e] : offr;
    const uint32_t eidx = 2u * offr + comp;  // float index of the operand inside its fibre
    const float* Ctf = reinterpret_cast<const float*>(Ct);
    const float* actf = reinterpret_cast<const float*>(act);
    const int srcbase = (int)(4u * (m >> 3) + kk);
    f32x4 D = {0.f, 0.f, 0.f, 0.f};
    // wave-uniform loop: every lane takes part in the matrix-core steps
    for (uint32_t fb = threadIdx.x & ~63u; fb < g.F; fb += (uint32_t)nt) {
        const uint32_t f = fb + lane;
        const bool valid = f < g.F;
        const uint32_t ph0 = valid ? g.base(a, j, f) : 0xffffffffu;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t p = (uint32_t)__shfl((int)ph0, 8 * u + srcbase, 64);
            float cvf = 0.f, avf = 0.f;
            if (p != 0xffffffffu && rlive) {
                cvf = Ctf[2u * p + eidx];
                avf = actf[2u * p + eidx];
            }
            D = __builtin_amdgcn_mfma_f32_16x16x4f32(cvf, avf, D, 0, 0, 0);
        }
        if (valid && store) {
            cf cv[B];
#pragma unroll
            for (int e = 0; e < B; ++e) cv[e] = Ct[ph0 + g.off[e]];
            block_digit_adj<cf, B, 1, 0>(cv, w);
#pragma unroll
            for (int e = 0; e < B; ++e) Ct[ph0 + g.off[e]] = cv[e];
        }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) Md[v] += (double)D[v];
}

// NT threads per work-group (256, 512 or 1024): the host picks the size
// whose resident waves are the most for the tile's LDS (a large tile leaves
// room for one or two work-groups per compute unit)
template <typename T, int B, int RD, int NT>
__global__ __launch_bounds__(NT) void gtt_bwd_block_kernel(BwdArgs ba) {
    using C = typename Tr<T>::C;
    using Acc = typename AccOf<C>::type;
    static_assert(RD >= 1 && RD == bwd_block_digits<C>(B), "digits per block");
    static_assert(NT % 64 == 0 && NT <= 1024 && (NT / 64) * B * B <= kThreads,
                  "the per-wave sums fit the reduction area (kThreads entries)");
    const PassArgs& a = ba.p;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const uint32_t rows = (uint32_t)a.P * (uint32_t)a.G;
    const uint32_t tileE = rows << a.logC;
    const uint32_t tileP = lds_tile_elems(tileE, a.pad_shift);
    const int wloc = ba.wloc;  // B * B
    // the layout of gtt_bwd_kernel: [acc][red][W][W^H][slots]
    unsigned char* pb = smem_raw;
    pb += bwd_align16((size_t)wloc * sizeof(Acc));
    Acc* red = reinterpret_cast<Acc*>(pb);
    pb += (size_t)kThreads * sizeof(Acc);
    pb += 2 * bwd_align16((size_t)wloc * sizeof(C));
    C* slot0 = reinterpret_cast<C*>(pb);
    auto slot = [&](int i) { return slot0 + (size_t)i * tileP; };
    const C* __restrict__ Wg = static_cast<const C*>(a.W);
    // W only (uniform: scalar registers); the adjoint passes read it
    // transposed and conjugated
    C w[B * B];
#pragma unroll
    for (int e = 0; e < B * B; ++e) w[e] = Wg[e];
    // complex radix 3 and 4: gradient sums on the matrix cores (FP64 sums of
    // the 16x16 FP32 blocks per lane); otherwise per-thread FP64 accumulators
    constexpr bool kMfmaGw = std::is_same<C, cf>::value && (B == 3 || B == 4) && RD == 1;
    Acc acc[kMfmaGw ? 1 : B * B];
#pragma unroll
    for (int e = 0; e < (kMfmaGw ? 1 : B * B); ++e) acc[e] = acc_zero(Acc{});
    [[maybe_unused]] double Md[4] = {0.0, 0.0, 0.0, 0.0};
    C* Ct = slot(1);
    // odd radices: element-wise tiles, addresses from the scalar walk
    constexpr bool kScalarWalk = (B & (B - 1)) != 0;
    for (int64_t t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
        tile_load<T, C, NT, kScalarWalk>(slot(0), a, static_cast<const T*>(a.in), t, rows);
        tile_load<T, C, NT, kScalarWalk>(Ct, a, static_cast<const T*>(ba.c_out), t, rows);
        __syncthreads();
        for (int o = 0; o < ba.nops; ++o) {
            const int op = ba.ops[o];
            const int kind = op & 3, blk = (op >> 2) & 63, src = (op >> 8) & 15, dst = (op >> 12) & 15;
            const int j0 = blk * RD;
            const int r = (a.k - j0) < RD ? (a.k - j0) : RD;
            if (kind == kOpFwd) {
                if constexpr (RD >= 4) { if (r == 4) { block_fwd<C, B, 4, NT>(slot(src), slot(dst), w, a, j0, rows); goto done; } }
                if constexpr (RD >= 3) { if (r == 3) { block_fwd<C, B, 3, NT>(slot(src), slot(dst), w, a, j0, rows); goto done; } }
                if constexpr (RD >= 2) { if (r == 2) { block_fwd<C, B, 2, NT>(slot(src), slot(dst), w, a, j0, rows); goto done; } }
                block_fwd<C, B, 1, NT>(slot(src), slot(dst), w, a, j0, rows);
            } else if (kind == kOpGw) {
                // the schedule puts the block's adjoint right after its
                // gradient sweep: both run here; the cotangent at the
                // group's input (block 0) only when it is stored
                const bool store = blk != 0 || a.out;
                if (o + 1 < ba.nops && (ba.ops[o + 1] & 3) == kOpAdj) ++o;
                if constexpr (RD >= 4) { if (r == 4) { block_gw_adj<C, Acc, B, 4, NT>(Ct, slot(src), w, acc, a, j0, rows, store); goto done; } }
                if constexpr (RD >= 3) { if (r == 3) { block_gw_adj<C, Acc, B, 3, NT>(Ct, slot(src), w, acc, a, j0, rows, store); goto done; } }
                if constexpr (RD >= 2) { if (r == 2) { block_gw_adj<C, Acc, B, 2, NT>(Ct, slot(src), w, acc, a, j0, rows, store); goto done; } }
                if constexpr (kMfmaGw)
                    block_gw_adj_cmfma<B>(Ct, slot(src), w, Md, a, j0, rows, store, NT);
                else
                    block_gw_adj<C, Acc, B, 1, NT>(Ct, slot(src), w, acc, a, j0, rows, store);
            }
            // (a lone adjoint never occurs: the host's schedules pair each
            // block's gradient sweep with its adjoint)
        done:
            __syncthreads();
        }
        if (a.out) tile_store<T, C, false, NT, kScalarWalk>(Ct, a, static_cast<T*>(a.out), t, rows);
        __syncthreads();
    }
    // work-group total, fixed order: lanes by a shuffle tree, then waves
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if constexpr (kMfmaGw) {
        // lane l holds D[4 (l / 16) + v][l % 16]: fold set 1's diagonal block
        // (lane l + 40) onto set 0's, then lane q < B forms gradient entry
        // (v, q), v < B: real part G[v][q] + G[4 + v][4 + q] (lanes q,
        // 20 + q), imaginary part G[4 + v][q] - G[v][4 + q] (lanes 16 + q,
        // 4 + q)
        double G8[4], re[4], im[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) G8[v] = Md[v] + __shfl_down(Md[v], 40, 64);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            re[v] = G8[v] + __shfl_down(G8[v], 20, 64);
            im[v] = __shfl_down(G8[v], 16, 64) - __shfl_down(G8[v], 4, 64);
        }
        if (lane < B) {
#pragma unroll
            for (int v = 0; v < B; ++v) red[wave * (B * B) + v * B + lane] = cd{re[v], im[v]};
        }
    } else {
#pragma unroll
        for (int e = 0; e < B * B; ++e) {
            Acc v = acc[e];
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) v = acc_add(v, acc_shfl_down(v, d));
            if (lane == 0) red[wave * (B * B) + e] = v;
        }
    }
    __syncthreads();
    Acc* part = static_cast<Acc*>(ba.partials) + (size_t)blockIdx.x * ba.wslot;
    for (int e = threadIdx.x; e < B * B; e += NT) {
        Acc v = red[e];
        for (int w_ = 1; w_ < NT / 64; ++w_) v = acc_add(v, red[w_ * (B * B) + e]);
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
template <typename K>
inline hipError_t bwd_launch_one(K kernel, const BwdArgs& a, unsigned grid, unsigned threads, size_t lds,
                                 hipStream_t s) {
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(threads), lds, s, a);
    return hipGetLastError();
}

// Resident waves per compute unit of a kernel at NT threads and `lds` bytes
// of LDS; 0 when it cannot run or spills to scratch.  Asked once per
// (kernel, NT, lds): the launches take it on every call.
template <typename K>
inline int bwd_resident_waves(K kernel, int nt, size_t lds) {
    static std::mutex mu;
    static std::map<std::tuple<const void*, int, size_t>, int> cache;
    const void* fp = reinterpret_cast<const void*>(kernel);
    const auto key = std::make_tuple(fp, nt, lds);
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    int waves = 0;
    hipFuncAttributes fa;
    if (hipFuncGetAttributes(&fa, fp) == hipSuccess && fa.localSizeBytes == 0 && fa.maxThreadsPerBlock >= nt &&
        (lds <= 65536 ||
         hipFuncSetAttribute(fp, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) == hipSuccess)) {
        int blocks = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kernel, nt, lds) == hipSuccess)
            waves = blocks * nt / 64;
    }
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = waves;
    return waves;
}

// the runtime-radix backward: the four-wave form (32-bit compute lanes, radix
// <= 16; where it does not spill) when more of its work-groups are resident at
// this LDS size, else the unconstrained one
template <typename T, int MAXB>
inline hipError_t launch_bwd_general(const BwdArgs& a, unsigned grid, size_t lds, hipStream_t s) {
    if constexpr (sizeof(typename Tr<T>::C) <= 8) {
        if (bwd_resident_waves(gtt_bwd_kernel<T, MAXB, true>, kThreads, lds) >
            bwd_resident_waves(gtt_bwd_kernel<T, MAXB, false>, kThreads, lds))
            return bwd_launch_one(gtt_bwd_kernel<T, MAXB, true>, a, grid, kThreads, lds, s);
    }
    return bwd_launch_one(gtt_bwd_kernel<T, MAXB, false>, a, grid, kThreads, lds, s);
}

// The register-block kernels of radix B at 256, 512 and 1024 threads (1024
// only where the per-wave sums fit the reduction area)
template <typename T, int B, int RD>
struct BwdBlockKernels {
    static constexpr bool k1024 = 16 * B * B <= kThreads;
    static auto get(int nt) {
        if (nt == 1024) return gtt_bwd_block_kernel<T, B, RD, k1024 ? 1024 : 512>;
        if (nt == 512) return gtt_bwd_block_kernel<T, B, RD, 512>;
        return gtt_bwd_block_kernel<T, B, RD, 256>;
    }
    // the work-group size with the most resident waves for this LDS
    // (ties: the smaller work-group)
    static int threads(size_t lds) {
        int best = kThreads, bw = bwd_resident_waves(get(kThreads), kThreads, lds);
        for (int nt : {512, 1024}) {
            if (nt == 1024 && !k1024) continue;
            const int w = bwd_resident_waves(get(nt), nt, lds);
            if (w > bw) {
                best = nt;
                bw = w;
            }
        }
        return best;
    }
};

// radix: 2..5 runs the register-block kernel of that radix (every digit uses
// the one W; the schedule counts blocks of bwd_block_digits digits), 16 / 32
// the matrix-core kernel (one W; 16-bit or float storage), 0 the
// runtime-radix kernel (radices up to maxb).  threads: the block kernel's
// work-group size (from launch_bwd_threads_t), ignored by the others.
template <typename T>
hipError_t launch_bwd_t(const BwdArgs& a, int maxb, int radix, unsigned grid, int threads, size_t lds,
                        hipStream_t s) {
    using C = typename Tr<T>::C;
    if (radix > 0) {
        constexpr int r2 = bwd_block_digits<C>(2), r3 = bwd_block_digits<C>(3), r4 = bwd_block_digits<C>(4),
                      r5 = bwd_block_digits<C>(5);
        switch (radix) {
            case 2: if constexpr (r2 > 0) return bwd_launch_one(BwdBlockKernels<T, 2, (r2 > 0 ? r2 : 1)>::get(threads), a, grid, threads, lds, s); break;
            case 3: if constexpr (r3 > 0) return bwd_launch_one(BwdBlockKernels<T, 3, (r3 > 0 ? r3 : 1)>::get(threads), a, grid, threads, lds, s); break;
            case 4: if constexpr (r4 > 0) return bwd_launch_one(BwdBlockKernels<T, 4, (r4 > 0 ? r4 : 1)>::get(threads), a, grid, threads, lds, s); break;
            case 5: if constexpr (r5 > 0) return bwd_launch_one(BwdBlockKernels<T, 5, (r5 > 0 ? r5 : 1)>::get(threads), a, grid, threads, lds, s); break;
            case 16: if constexpr (bwd_mfma_ok<T>()) return bwd_launch_one(gtt_bwd_mfma_kernel<T, 16>, a, grid, kThreads, lds, s); break;
            case 32: if constexpr (bwd_mfma_ok<T>()) return bwd_launch_one(gtt_bwd_mfma_kernel<T, 32>, a, grid, kThreads, lds, s); break;
            default: break;
        }
        return hipErrorInvalidValue;
    }
    if (maxb <= 8) return launch_bwd_general<T, 8>(a, grid, lds, s);
    if (maxb <= 16) return launch_bwd_general<T, 16>(a, grid, lds, s);
    if (maxb <= 32) return bwd_launch_one(gtt_bwd_kernel<T, 32>, a, grid, kThreads, lds, s);
    return hipErrorInvalidValue;
}

// work-group size of the register-block kernel of this radix for `lds`
// bytes of LDS (kThreads for the runtime-radix kernel)
template <typename T>
int launch_bwd_threads_t(int radix, size_t lds) {
    using C = typename Tr<T>::C;
    constexpr int r2 = bwd_block_digits<C>(2), r3 = bwd_block_digits<C>(3), r4 = bwd_block_digits<C>(4),
                  r5 = bwd_block_digits<C>(5);
    switch (radix) {
        case 2: if constexpr (r2 > 0) return BwdBlockKernels<T, 2, (r2 > 0 ? r2 : 1)>::threads(lds); break;
        case 3: if constexpr (r3 > 0) return BwdBlockKernels<T, 3, (r3 > 0 ? r3 : 1)>::threads(lds); break;
        case 4: if constexpr (r4 > 0) return BwdBlockKernels<T, 4, (r4 > 0 ? r4 : 1)>::threads(lds); break;
        case 5: if constexpr (r5 > 0) return BwdBlockKernels<T, 5, (r5 > 0 ? r5 : 1)>::threads(lds); break;
        default: break;
    }
    return kThreads;
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
    hipError_t launch_bwd_##NAME(const BwdArgs& a, int maxb, int radix, unsigned grid, int threads,      \
                                 size_t lds, hipStream_t s) {                                            \
        return launch_bwd_t<T>(a, maxb, radix, grid, threads, lds, s);                                   \
    }                                                                                                    \
    int launch_bwd_threads_##NAME(int radix, size_t lds) { return launch_bwd_threads_t<T>(radix, lds); }  \
    int bwd_block_digits_##NAME(int b) { return bwd_block_digits<typename Tr<T>::C>(b); }              \
    hipError_t launch_reduce_##NAME(const void* partials, int64_t nparts, int bb, void* out,            \
                                    hipStream_t s) {                                                     \
        return launch_reduce_t<T>(partials, nparts, bb, out, s);                                         \
    }                                                                                                    \
    }
