// Complex radix-8 digit passes and weight gradient on the FP32 matrix cores.
//
// A complex 8 x 8 product y = W x is the real 16 x 16 product
//     [Re y; Im y] = [[Re W, -Im W], [Im W, Re W]] [Re x; Im x],
// which is one 16x16 MFMA block.  With v_mfma_f32_16x16x4_f32, K is split in
// four slices of four; rows and columns of the real matrix are ordered so that
// every lane sees complex values in the interleaved (re, im) memory layout:
//   B operand, K slice kk: lane (q = l/16, fibre i = l%16) holds component
//     kk & 1 of element 2q + (kk >> 1) of fibre i, i.e. over the four slices
//     the lane supplies x[2q].re, x[2q].im, x[2q+1].re, x[2q+1].im;
//   result: lane (q, i) holds y[2q].re, y[2q].im, y[2q+1].re, y[2q+1].im.
// So one wave reads two complex elements per lane from LDS, runs four MFMAs
// and writes two complex results back in place (16 fibres per wave step).
//
// The weight gradient sum_f c_f a_f^H over the fibres of a digit is the real
// 16 x 16 product M = [c]_{16 x F} [a]^T_{F x 16} accumulated over fibres
// (K = fibres, four per MFMA), with row index m = 2e + comp for element e:
//   Re gW[r][q] = M[2r][2q] + M[2r+1][2q+1],  Im gW[r][q] = M[2r+1][2q] - M[2r][2q+1].
// Every digit of every group adds into the same gradient, so one accumulator
// per wave collects all of them: the FP32 MFMA chain covers one digit of one
// tile (at most a few hundred terms), and is then added into an FP64
// accumulator, which bounds the rounding error of long sums; the work-group
// total is rounded to FP32 once.
#pragma once

#include <type_traits>

#include "gtt_args.hpp"
#include "gtt_pass.hpp"
#include "gtt_types.hpp"

namespace gtt {

typedef float f32x4_c __attribute__((ext_vector_type(4)));

struct CFrag8 {
    float a[4];  // A operand of the four K slices
};

// real 16 x 16 block of W (or W^H) at (m, k) in the interleaved ordering
__device__ __forceinline__ float creal_block(const cf* __restrict__ W, int adjoint, int m, int k) {
    const int e_out = 2 * (m >> 2) + ((m & 3) >> 1), c_out = m & 1;
    const int e_in = 2 * (k & 3) + (k >> 3), c_in = (k >> 2) & 1;
    cf w = adjoint ? cconj(W[e_in * 8 + e_out]) : W[e_out * 8 + e_in];
    if (c_out == 0) return c_in == 0 ? w.re : -w.im;
    return c_in == 0 ? w.im : w.re;
}

__device__ __forceinline__ void load_cfrag8(CFrag8& f, const cf* __restrict__ W, int adjoint) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) f.a[kk] = creal_block(W, adjoint, lane & 15, 4 * kk + (lane >> 4));
}

// tile position of element 0 of fibre f of digit j (radix 8: b^j = 2^(3j))
__device__ __forceinline__ uint32_t fibre_base(const PassArgs& a, int j, uint32_t f) {
    const uint32_t Cm = (1u << a.logC) - 1u;
    const uint32_t c = f & Cm;
    const uint32_t f1 = f >> a.logC;
    const uint32_t lo = f1 & ((1u << (3 * j)) - 1u);
    const uint32_t Q = f1 >> (3 * j);
    return ((Q << (3 * j + 3)) + lo) << a.logC | c;
}

// W (fragments f) along digit j of every fibre of the complex tile: reads
// src, writes dst (in place when they are equal).  NT threads per work-group.
template <int NT = kThreads>
__device__ __forceinline__ void cmfma_stage8(const cf* src, cf* dst, const PassArgs& a, int j, uint32_t rows,
                                             const CFrag8& fr) {
    const uint32_t F = (rows << a.logC) >> 3;
    const uint32_t step = (uint32_t)a.bpow[j] << a.logC;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int q = lane >> 4;
    const uint32_t ngrp = (F + 15) >> 4;
    for (uint32_t grp = wave; grp < ngrp; grp += NT / 64) {
        const uint32_t f = (grp << 4) + (lane & 15);
        const bool valid = f < F;
        uint32_t p0 = 0, p1 = 0;
        cf x0 = {0.f, 0.f}, x1 = {0.f, 0.f};
        if (valid) {
            const uint32_t lam0 = fibre_base(a, j, f);
            p0 = lds_phys(lam0 + (2 * q) * step, a.pad_shift);
            p1 = lds_phys(lam0 + (2 * q + 1) * step, a.pad_shift);
            x0 = src[p0];
            x1 = src[p1];
        }
        f32x4_c acc = {0.f, 0.f, 0.f, 0.f};
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(fr.a[0], x0.re, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(fr.a[1], x0.im, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(fr.a[2], x1.re, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(fr.a[3], x1.im, acc, 0, 0, 0);
        if (valid) {
            dst[p0] = cf{acc[0], acc[1]};
            dst[p1] = cf{acc[2], acc[3]};
        }
    }
}

// M += sum over the fibres of digit j of [c] [a]^T (see the header comment).
template <int NT = kThreads>
__device__ __forceinline__ void cmfma_gw8(const cf* ct, const cf* at, const PassArgs& a, int j, uint32_t rows,
                                          f32x4_c& M) {
    const uint32_t F = (rows << a.logC) >> 3;
    const uint32_t step = (uint32_t)a.bpow[j] << a.logC;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int m = lane & 15;
    const int e = m >> 1;
    const bool im = (m & 1) != 0;
    const uint32_t ngrp = (F + 3) >> 2;
    const float* ctf = reinterpret_cast<const float*>(ct);
    const float* atf = reinterpret_cast<const float*>(at);
    for (uint32_t grp = wave; grp < ngrp; grp += NT / 64) {
        const uint32_t f = (grp << 2) + (lane >> 4);
        float cv = 0.f, av = 0.f;
        if (f < F) {
            const uint32_t ph = lds_phys(fibre_base(a, j, f) + e * step, a.pad_shift);
            cv = ctf[2 * ph + im];
            av = atf[2 * ph + im];
        }
        M = __builtin_amdgcn_mfma_f32_16x16x4f32(cv, av, M, 0, 0, 0);
    }
}


__global__ __launch_bounds__(kThreads) void gtt_c64_mfma8_pass_kernel(PassArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cf* lds = reinterpret_cast<cf*>(smem_raw);
    CFrag8 fr;
    load_cfrag8(fr, static_cast<const cf*>(a.W), a.adjoint);
    tile_loop<cf, cf>(lds, a, [&](cf* t, uint32_t rows, int64_t) {
        for (int j = 0; j < a.k; ++j) {
            cmfma_stage8(t, t, a, j, rows, fr);
            __syncthreads();
        }
        return false;
    });
}

// Backward of one digit group (k <= 4 digits), complex radix 8, on the
// matrix cores, kBwdThreads threads (the LDS of one group tile allows one
// work-group per compute unit; 16 waves keep the MFMA and LDS pipes busy).
// LDS holds the group input A, two activation slots T1, T2 and the
// cotangent Ct.  With a_s the input of the pass on digit s:
//   T1 = a_1; T2 = a_2 (then a_3 = W T2 in place when k = 4);
//   for s = k-1 .. 0: accumulate the c a_s^H sums, then Ct <- W^H Ct along s,
//   recomputing a_2 from T1 once when k = 4.
// The next tile's A and Ct are fetched into registers while the current tile
// is processed.
constexpr int kBwdThreads = 1024;
constexpr int kBwdVec = 4;  // 16-byte vectors per thread and buffer (tile <= 8192 c64)

// NV 16-byte vectors per thread and buffer; FULL: the tile has exactly
// NV * kBwdThreads vectors (no bounds test)
template <int NV = kBwdVec, bool FULL = false>
__device__ __forceinline__ void bwd_fetch(uint4 (&buf)[NV], const PassArgs& a, const cf* __restrict__ in,
                                          int64_t t, uint32_t tileE) {
    const bool contig = a.mode == kContigVec;
    const int64_t hb = contig ? 0 : tile_hb(a, t);
    const int64_t l = contig ? 0 : t - hb * a.L;
    const uint32_t nvec = tileE / 2;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const uint32_t i = threadIdx.x + v * kBwdThreads;
        if (FULL || i < nvec) buf[v] = *reinterpret_cast<const uint4*>(in + vec_offset<cf>(a, t, i, hb, l, tileE));
    }
}

template <int NV = kBwdVec, bool FULL = false>
__device__ __forceinline__ void bwd_commit(cf* lds, const uint4 (&buf)[NV], const PassArgs& a, uint32_t tileE) {
    const uint32_t nvec = tileE / 2;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const uint32_t i = threadIdx.x + v * kBwdThreads;
        if (FULL || i < nvec) {
            cf vals[2];
            *reinterpret_cast<uint4*>(vals) = buf[v];
            const uint32_t ph = lds_phys(i * 2, a.pad_shift);
            lds[ph] = vals[0];
            lds[ph + 1] = vals[1];
        }
    }
}

__device__ __forceinline__ void bwd_store(const cf* lds, const PassArgs& a, cf* __restrict__ out, int64_t t,
                                          uint32_t tileE) {
    const bool contig = a.mode == kContigVec;
    const int64_t hb = contig ? 0 : tile_hb(a, t);
    const int64_t l = contig ? 0 : t - hb * a.L;
    const uint32_t nvec = tileE / 2;
    for (uint32_t i = threadIdx.x; i < nvec; i += kBwdThreads) {
        cf vals[2];
        const uint32_t ph = lds_phys(i * 2, a.pad_shift);
        vals[0] = lds[ph];
        vals[1] = lds[ph + 1];
        *reinterpret_cast<uint4*>(out + vec_offset<cf>(a, t, i, hb, l, tileE)) = *reinterpret_cast<const uint4*>(vals);
    }
}

__global__ __launch_bounds__(kBwdThreads) void gtt_c64_mfma8_bwd_kernel(CBwdArgs ba) {
    const PassArgs& a = ba.p;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const uint32_t rows = (uint32_t)a.P * (uint32_t)a.G;
    const uint32_t tileE = rows << a.logC;
    const uint32_t tileP = lds_tile_elems(tileE, a.pad_shift);
    cf* A = reinterpret_cast<cf*>(smem_raw);
    cf* T1 = A + tileP;
    cf* Ct = T1 + tileP;
    cf* T2 = Ct + tileP;  // used only when the group has three or more digits
    // 16 waves x 256 doubles for the final reduction, reusing the tiles' LDS
    double* red = reinterpret_cast<double*>(smem_raw);
    CFrag8 fw, fh;
    load_cfrag8(fw, static_cast<const cf*>(a.W), 0);
    load_cfrag8(fh, static_cast<const cf*>(a.W), 1);
    double Md[4] = {0.0, 0.0, 0.0, 0.0};
    const cf* xin = static_cast<const cf*>(a.in);
    const cf* cin = static_cast<const cf*>(ba.c_out);
    uint4 pa[kBwdVec], pc[kBwdVec];
    int64_t t = blockIdx.x;
    if (t < a.ntiles) {
        bwd_fetch(pa, a, xin, t, tileE);
        bwd_fetch(pc, a, cin, t, tileE);
    }
    auto gw = [&](const cf* act, int s) {
        f32x4_c M = {0.f, 0.f, 0.f, 0.f};
        cmfma_gw8<kBwdThreads>(Ct, act, a, s, rows, M);
#pragma unroll
        for (int v = 0; v < 4; ++v) Md[v] += (double)M[v];
        __syncthreads();  // every wave has read Ct before the pass on s rewrites it
    };
    auto adj = [&](int s) {
        cmfma_stage8<kBwdThreads>(Ct, Ct, a, s, rows, fh);
        __syncthreads();
    };
    for (; t < a.ntiles; t += gridDim.x) {
        bwd_commit(A, pa, a, tileE);
        bwd_commit(Ct, pc, a, tileE);
        __syncthreads();
        const int64_t tn = t + gridDim.x;
        if (tn < a.ntiles) {  // in flight while this tile is processed
            bwd_fetch(pa, a, xin, tn, tileE);
            bwd_fetch(pc, a, cin, tn, tileE);
        }
        const int k = a.k;
        if (k >= 2) {
            cmfma_stage8<kBwdThreads>(A, T1, a, 0, rows, fw);  // a_1
            __syncthreads();
        }
        if (k >= 3) {
            cmfma_stage8<kBwdThreads>(T1, T2, a, 1, rows, fw);  // a_2
            __syncthreads();
        }
        if (k == 4) {
            cmfma_stage8<kBwdThreads>(T2, T2, a, 2, rows, fw);  // a_3
            __syncthreads();
            gw(T2, 3);
            adj(3);
            cmfma_stage8<kBwdThreads>(T1, T2, a, 1, rows, fw);  // a_2 again
            __syncthreads();
        }
        if (k >= 3) {
            gw(T2, 2);
            adj(2);
        }
        if (k >= 2) {
            gw(T1, 1);
            adj(1);
        }
        gw(A, 0);
        // out is null for the first digit group when only gW is wanted
        if (a.out) {
            adj(0);
            bwd_store(Ct, a, static_cast<cf*>(a.out), t, tileE);
        }
        __syncthreads();
    }
    // reduce the waves' 16 x 16 blocks in a fixed order, then form the
    // complex gradient
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < 4; ++v) red[wave * 256 + (4 * (lane >> 4) + v) * 16 + (lane & 15)] = Md[v];
    __syncthreads();
    if (threadIdx.x < 64) {
        const int r = threadIdx.x >> 3, q = threadIdx.x & 7;
        auto Mv = [&](int mm, int nn) {
            double s = 0.0;
            for (int w = 0; w < kBwdThreads / 64; ++w) s += red[w * 256 + mm * 16 + nn];
            return s;
        };
        cd g;
        g.re = Mv(2 * r, 2 * q) + Mv(2 * r + 1, 2 * q + 1);
        g.im = Mv(2 * r + 1, 2 * q) - Mv(2 * r, 2 * q + 1);
        static_cast<cd*>(ba.partials)[(size_t)blockIdx.x * 64 + threadIdx.x] = g;
    }
}


// ---------------------------------------------------------------------------
// Radix-8 passes and backward with per-lane LDS addresses (tiles of 2048 * NI
// complex64 elements, K <= 4 digits, 1024 threads).
//
// A tile position is a bit string: column bits (logC), three bits per digit,
// then row bits.  The LDS padding adds x >> p for a few shifts p, and a shift
// of a sum of numbers with disjoint bits is the sum of their shifts, so
// phys(u | v) = phys(u) + phys(v) when u & v == 0.  Element e of fibre f of
// digit j sits at dep_j(f) | e << h_j, where dep_j inserts three zero bits at
// h_j = logC + 3 j; dep_j is additive over disjoint bits too.  Splitting the
// fibre index into a lane part and a loop part with disjoint bits therefore
// splits every LDS address into a per-lane base (registers, once per launch)
// plus an offset that is the same for the whole work-group.
//
// Fibres of a digit: F = 256 NI; bit 8 is the loop step it.  The planner
// picks per digit an 8-bit mask (PassArgs::fmap): in step it, wave w owns the
// 16 fibres whose bits outside the mask spell w.  In the pass, lane (q, i)
// handles elements 2q, 2q+1 of the fibre whose mask bits spell i.  In the
// gradient sums, lane group k (0..3) sets fibre bits kb0 (k & 1) and kb1
// (k >> 1), and the four MFMAs of a block run over the other two mask bits;
// so a wave reads for the sums exactly the fibres its own pass rewrites next
// and the two need no barrier in between.  The planner chooses the padding
// and the maps so that these accesses avoid LDS bank conflicts.
__device__ __forceinline__ uint32_t digit_deposit(uint32_t v, uint32_t h) {
    return ((v >> h) << (h + 3)) | (v & ((1u << h) - 1u));
}

// the low bits of v placed, in order, at the set bits of mask (8 bits)
__device__ __forceinline__ uint32_t deposit8(uint32_t v, uint32_t mask) {
    uint32_t r = 0;
#pragma unroll
    for (int b = 0; b < 8; ++b)
        if (mask >> b & 1u) {
            r |= (v & 1u) << b;
            v >>= 1;
        }
    return r;
}

template <int V>
using IntC = std::integral_constant<int, V>;

struct DigitMap {
    uint32_t mask, kb0, kb1, ob0, ob1;
};

__device__ __forceinline__ DigitMap digit_map(uint64_t fmap, int j) {
    const uint32_t code = (uint32_t)(fmap >> (16 * j)) & 0xffffu;
    DigitMap d;
    d.mask = code & 0xffu;
    d.kb0 = (code >> 8) & 7u;
    d.kb1 = (code >> 11) & 7u;
    const uint32_t rest = d.mask & ~(1u << d.kb0) & ~(1u << d.kb1);
    d.ob0 = __builtin_ctz(rest);
    d.ob1 = __builtin_ctz(rest & (rest - 1u));
    return d;
}

// W (fragments fr) along the digit whose three bits start at h, over all
// fibres of a 2048 * NI element tile: lane (q, i) takes elements 2q, 2q+1 of
// its fibre of step it at byte offsets p0, p1 plus the step's uniform
// offset.  src -> dst, in place when equal.
template <int NI>
struct PassRegs {
    cf x0[NI], x1[NI];
};

template <int NI>
__device__ __forceinline__ void cpass8_load(PassRegs<NI>& r, const unsigned char* src, uint32_t p0, uint32_t p1,
                                            uint32_t h, int pad) {
#pragma unroll
    for (int it = 0; it < NI; ++it) {
        const uint32_t so = lds_phys(digit_deposit(256u * it, h), pad) * 8u;
        r.x0[it] = *reinterpret_cast<const cf*>(src + p0 + so);
        r.x1[it] = *reinterpret_cast<const cf*>(src + p1 + so);
        __builtin_amdgcn_sched_barrier(0);
    }
}

// step by step: the MFMA chain of a step and its stores, then the next
// step (whose loads may still be in flight while the first one computes)
template <int NI>
__device__ __forceinline__ void cpass8_compute_store(const PassRegs<NI>& r, unsigned char* dst, uint32_t p0,
                                                     uint32_t p1, uint32_t h, int pad, const CFrag8& fr) {
#pragma unroll
    for (int it = 0; it < NI; ++it) {
        __builtin_amdgcn_sched_barrier(0);
        f32x4_c acc = {0.f, 0.f, 0.f, 0.f};
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(fr.a[0], r.x0[it].re, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(fr.a[1], r.x0[it].im, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(fr.a[2], r.x1[it].re, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(fr.a[3], r.x1[it].im, acc, 0, 0, 0);
        const uint32_t so = lds_phys(digit_deposit(256u * it, h), pad) * 8u;
        *reinterpret_cast<cf*>(dst + p0 + so) = cf{acc[0], acc[1]};
        *reinterpret_cast<cf*>(dst + p1 + so) = cf{acc[2], acc[3]};
    }
}

// as above, keeping the results in registers (out)
template <int NI>
__device__ __forceinline__ void cpass8_compute_store_keep(const PassRegs<NI>& r, unsigned char* dst, uint32_t p0,
                                                          uint32_t p1, uint32_t h, int pad, const CFrag8& fr,
                                                          f32x4_c (&out)[NI]) {
#pragma unroll
    for (int it = 0; it < NI; ++it) {
        __builtin_amdgcn_sched_barrier(0);
        f32x4_c acc = {0.f, 0.f, 0.f, 0.f};
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(fr.a[0], r.x0[it].re, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(fr.a[1], r.x0[it].im, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(fr.a[2], r.x1[it].re, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(fr.a[3], r.x1[it].im, acc, 0, 0, 0);
        const uint32_t so = lds_phys(digit_deposit(256u * it, h), pad) * 8u;
        *reinterpret_cast<cf*>(dst + p0 + so) = cf{acc[0], acc[1]};
        *reinterpret_cast<cf*>(dst + p1 + so) = cf{acc[2], acc[3]};
        out[it] = acc;
    }
}

// W (fragments fr) along the digit whose three bits start at h, over all
// fibres of a 2048 * NI element tile: lane (q, i) takes elements 2q, 2q+1 of
// its fibre of step it at byte offsets p0, p1 plus the step's uniform
// offset.  src -> dst, in place when equal.  All loads are issued before the
// first MFMA, so the phase waits for LDS once.
template <int NI>
__device__ __forceinline__ void cpass8(const unsigned char* src, unsigned char* dst, uint32_t p0, uint32_t p1,
                                       uint32_t h, int pad, const CFrag8& fr) {
    PassRegs<NI> r;
    cpass8_load<NI>(r, src, p0, p1, h, pad);
    __builtin_amdgcn_sched_barrier(0);
    cpass8_compute_store<NI>(r, dst, p0, p1, h, pad, fr);
}

// per-lane byte offsets of the pass elements 2q, 2q+1 for digits 0..K-1
template <int K>
__device__ __forceinline__ void cpass8_lane_offsets(uint32_t (&P0)[K], uint32_t (&P1)[K], uint64_t fmap, int logC,
                                                    int pad) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t hi = (uint32_t)(lane >> 4), lo = (uint32_t)(lane & 15);
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const DigitMap d = digit_map(fmap, j);
        const uint32_t h = (uint32_t)logC + 3u * j;
        const uint32_t f = deposit8((uint32_t)wave, ~d.mask & 0xffu) | deposit8(lo, d.mask);
        const uint32_t L0 = digit_deposit(f, h) | ((2u * hi) << h);
        P0[j] = lds_phys(L0, pad) * 8u;
        P1[j] = lds_phys(L0 | (1u << h), pad) * 8u;
    }
}

// LDS layout parameters of a launch: from the arguments, or fixed at compile
// time for the layouts the planner produces for common shapes, so that
// every uniform LDS offset becomes an instruction immediate
struct LayoutArgs {
    static constexpr bool kFixed = false;
    static constexpr uint32_t kPmap = 0;  // runtime layouts keep every barrier
    __device__ static int pad(const PassArgs& a) { return a.pad_shift; }
    __device__ static int logc(const PassArgs& a) { return a.logC; }
    __device__ static uint64_t fmap(const PassArgs& a) { return a.fmap; }
};
template <int PAD, int LOGC, uint64_t FMAP, uint32_t PMAP = 0>
struct LayoutFixed {
    static constexpr bool kFixed = true;
    static constexpr int kPad = PAD, kLogC = LOGC;
    static constexpr uint64_t kFmap = FMAP;
    static constexpr uint32_t kPmap = PMAP;  // paired layout: pass-only maps of digits 1, 2
    __device__ static int pad(const PassArgs&) { return PAD; }
    __device__ static int logc(const PassArgs&) { return LOGC; }
    __device__ static uint64_t fmap(const PassArgs&) { return FMAP; }
};

// Non-temporal tile I/O for the compiled layouts where it measured faster:
// strided tiles in the forward pass, every backward tile
template <class LAY>
constexpr bool nt_pass_io() {
    if constexpr (LAY::kFixed) return LAY::kLogC > 0;
    else return false;
}
template <class LAY>
constexpr bool nt_bwd_io() {
    return LAY::kFixed;
}

// Tile transfers: 16-byte global accesses (two elements per lane and
// access), two 64-bit LDS accesses.  NV = tileE / 2048 vectors per thread.
// A thread's global offsets relative to the tile origin and its LDS offsets
// are the same for every tile; only the origin changes, and the walk over
// the work-group's tiles (t += gridDim.x) updates it without divisions.
// position of a work-group's current tile in the walk t += gridDim.x
struct TileCursor {
    int64_t origin;  // element offset of the tile's origin
    int64_t hb, l;   // strided tiles: hi block and column block
};

template <int NV, bool NT = false>
struct TileWalk {
    int64_t goff[NV];   // elements from the tile origin to this thread's vector v
    uint32_t loff[NV];  // LDS byte offset of that vector's first element
    int64_t dq, dr;     // gridDim.x = dq * L + dr (strided tiles)
    int64_t span;       // elements per hi block (G * S, strided tiles)

    __device__ __forceinline__ TileCursor init(const PassArgs& a, uint32_t tileE, int pad) {
        const bool contig = a.mode == kContigVec;
        const int lcv = a.logC - 1;  // log2(vectors per row)
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const uint32_t i = threadIdx.x + v * kBwdThreads;
            goff[v] = contig ? (int64_t)i * 2
                             : (int64_t)(i >> lcv) * a.S + (int64_t)(i & ((1u << lcv) - 1u)) * 2;
            loff[v] = lds_phys(2u * i, pad) * 8u;
        }
        span = (int64_t)a.G * a.S;
        const int64_t t = blockIdx.x;
        TileCursor c;
        if (contig) {
            c.origin = t * (int64_t)tileE;
            c.hb = c.l = dq = dr = 0;
        } else {
            c.hb = t / a.L;
            c.l = t - c.hb * a.L;
            dq = (int64_t)gridDim.x / a.L;
            dr = (int64_t)gridDim.x - dq * a.L;
            c.origin = c.hb * span + (c.l << a.logC);
        }
        return c;
    }
    // the work-group's next tile (t + gridDim.x)
    __device__ __forceinline__ TileCursor next(const PassArgs& a, uint32_t tileE, TileCursor c) const {
        if (a.mode == kContigVec) {
            c.origin += (int64_t)gridDim.x * tileE;
        } else {
            c.l += dr;
            c.hb += dq;
            if (c.l >= a.L) {
                c.l -= a.L;
                c.hb += 1;
            }
            c.origin = c.hb * span + (c.l << a.logC);
        }
        return c;
    }
    __device__ __forceinline__ void fetch(uint4 (&buf)[NV], const cf* __restrict__ in, const TileCursor& c) const {
#pragma unroll
        for (int v = 0; v < NV; ++v) buf[v] = gload16<NT>(in + c.origin + goff[v]);
    }
    __device__ __forceinline__ void commit(unsigned char* lds, const uint4 (&buf)[NV]) const {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            cf vals[2];
            *reinterpret_cast<uint4*>(vals) = buf[v];
            // a pair never straddles a pad (shifts >= 1): consecutive slots
            *reinterpret_cast<cf*>(lds + loff[v]) = vals[0];
            *reinterpret_cast<cf*>(lds + loff[v] + 8) = vals[1];
        }
    }
    __device__ __forceinline__ void store(const unsigned char* lds, cf* __restrict__ out, const TileCursor& c) const {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            cf vals[2];
            vals[0] = *reinterpret_cast<const cf*>(lds + loff[v]);
            vals[1] = *reinterpret_cast<const cf*>(lds + loff[v] + 8);
            gstore16<NT>(out + c.origin + goff[v], *reinterpret_cast<const uint4*>(vals));
        }
    }
};

// Forward (or adjoint) pass of K <= 4 radix-8 digits on tiles of 2048 * NI
// complex64 elements; the next tile is fetched into registers while the
// current one runs its digit passes.
// (two work-groups per compute unit: eight waves per SIMD, at most 64 VGPRs)
template <int K, int NI, class LAY>
__global__ __launch_bounds__(kBwdThreads, 8) void gtt_c64_mfma8_pass_fast_kernel(PassArgs a) {
    static_assert(K >= 1 && K <= 4 && NI >= 1 && NI <= 2, "tile shape");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr uint32_t tileE = 2048u * NI;
    constexpr int NE = NI;  // 16-byte vectors per thread
    const int pad = LAY::pad(a);
    const int logC = LAY::logc(a);
    uint32_t P0[K], P1[K];
    cpass8_lane_offsets<K>(P0, P1, LAY::fmap(a), logC, pad);
    CFrag8 fr;
    load_cfrag8(fr, static_cast<const cf*>(a.W), a.adjoint);
    const cf* in = static_cast<const cf*>(a.in);
    cf* out = static_cast<cf*>(a.out);
    uint4 pa[NE];
    TileWalk<NE, nt_pass_io<LAY>()> tw;
    TileCursor cur = tw.init(a, tileE, pad);
    int64_t t = blockIdx.x;
    if (t < a.ntiles) tw.fetch(pa, in, cur);
    for (; t < a.ntiles; t += gridDim.x) {
        // keep base + offset sums inside the loop: hoisted, they would hold
        // one register per (digit, step)
#pragma unroll
        for (int j = 0; j < K; ++j) asm volatile("" : "+v"(P0[j]), "+v"(P1[j]));
        tw.commit(smem_raw, pa);
        __syncthreads();
        const TileCursor nxt = tw.next(a, tileE, cur);
        if (t + gridDim.x < a.ntiles) tw.fetch(pa, in, nxt);
#pragma unroll
        for (int j = 0; j < K; ++j) {
            cpass8<NI>(smem_raw, smem_raw, P0[j], P1[j], (uint32_t)logC + 3u * j, pad, fr);
            __syncthreads();
        }
        tw.store(smem_raw, out, cur);
        __syncthreads();
        cur = nxt;
    }
}

// Backward of one digit group.  LDS holds the cotangent Ct, the group input
// A and activation slots T1, T2 (a_s = input of the pass on digit s).  K = 4:
//   T1 = a_1; T2 = a_2; T1 = a_3;  digit 3: sums + adjoint;
//   digit 2 (reads T2, Ct) in the same phase as T1 = a_1 recomputed from A;
//   digit 1 (T1); digit 0 (A).
// K = 3 keeps a_1, a_2; K = 2 keeps a_1.  In the gradient sums, row
// m = 8 comp + e of the real 16 x 16 block is component comp of element e.
//
// D0 (contiguous tiles whose digit 0 has stride 1): a lane's two pass
// elements of a digit-0 fibre are 16 contiguous bytes in global memory, and
// every fibre is one aligned 64-byte segment.  The group input is then
// loaded straight in the digit-0 pass layout, so a_1 is computed from the
// registers in the phase that stores A (and kept there: K = 4 writes it
// back into T1 instead of recomputing it), and the adjoint pass of digit 0
// writes gx straight to global memory: two phases and their LDS round trips
// fewer per tile.
template <int K, int NI, class LAY, bool D0 = false>
__global__ __launch_bounds__(kBwdThreads) void gtt_c64_mfma8_bwd_fast_kernel(CBwdArgs ba) {
    static_assert(K >= 1 && K <= 4 && NI >= 1 && NI <= 2, "tile shape");
    static_assert(!D0 || (K >= 2 && LAY::kFixed), "direct digit-0 I/O: fixed layouts, two digits or more");
    const PassArgs& a = ba.p;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr uint32_t tileE = 2048u * NI;
    constexpr int NE = NI;  // 16-byte vectors per thread
    const int pad = LAY::pad(a);
    const int logC = LAY::logc(a);
    const uint64_t fmap = LAY::fmap(a);
    const uint32_t tileB = lds_tile_elems(tileE, pad) * (uint32_t)sizeof(cf);
    // the most used tiles first: their offsets fit instruction immediates
    unsigned char* Cb = smem_raw;
    unsigned char* T1b = Cb + tileB;
    unsigned char* T2b = Cb + 2u * tileB;  // K >= 3 only
    unsigned char* Ab = Cb + (K >= 3 ? 3u : K == 2 ? 2u : 1u) * tileB;
    double* red = reinterpret_cast<double*>(smem_raw);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t hi = (uint32_t)(lane >> 4), lo = (uint32_t)(lane & 15);
    uint32_t P0[K], P1[K], GB[K];
    cpass8_lane_offsets<K>(P0, P1, fmap, logC, pad);
    // Paired layout (four digits, direct digit-0 I/O): the recomputing passes
    // of digits 1 and 2 run on their own maps, under which every wave owns
    // whole digit-1 x digit-2 blocks, and the fused phases of digits 1 and 0
    // on maps under which every wave owns whole digit-0 x digit-1 blocks.
    // The second phase of each pair reads only what its own wave wrote in
    // the first, so the pair needs no work-group barrier in between: five
    // barriers per tile instead of seven.
    constexpr bool kPair = D0 && K == 4 && LAY::kPmap != 0;
    [[maybe_unused]] uint32_t Q0[2], Q1[2];
    if constexpr (kPair) {
        const int lane_ = threadIdx.x & 63, wave_ = threadIdx.x >> 6;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const uint32_t mask = (LAY::kPmap >> (8 * i)) & 0xffu, h = 3u * (uint32_t)(i + 1);
            const uint32_t f = deposit8((uint32_t)wave_, ~mask & 0xffu) | deposit8((uint32_t)(lane_ & 15), mask);
            const uint32_t L0 = digit_deposit(f, h) | ((2u * (uint32_t)(lane_ >> 4)) << h);
            Q0[i] = lds_phys(L0, pad) * 8u;
            Q1[i] = lds_phys(L0 | (1u << h), pad) * 8u;
        }
    }
    // between the two phases of a pair: the wave's own LDS writes ordered
    // before its reads (no other wave's data is involved)
    auto wave_sync = [&]() {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const DigitMap d = digit_map(fmap, j);
        const uint32_t h = (uint32_t)logC + 3u * j;
        const uint32_t f = deposit8((uint32_t)wave, ~d.mask & 0xffu) | ((hi & 1u) << d.kb0) | ((hi >> 1) << d.kb1);
        GB[j] = lds_phys(digit_deposit(f, h) | ((lo & 7u) << h), pad) * 8u + 4u * (lo >> 3);
    }
    // uniform offset of gradient MFMA t of digit j
    auto goff = [&](int j, int t) {
        const DigitMap d = digit_map(fmap, j);
        const uint32_t u = (uint32_t)(t & 3);
        const uint32_t f = 256u * (uint32_t)(t >> 2) | ((u & 1u) << d.ob0) | ((u >> 1) << d.ob1);
        return lds_phys(digit_deposit(f, (uint32_t)logC + 3u * j), pad) * 8u;
    };
    CFrag8 fw, fh;
    load_cfrag8(fw, static_cast<const cf*>(a.W), 0);
    load_cfrag8(fh, static_cast<const cf*>(a.W), 1);
    double Md[4] = {0.0, 0.0, 0.0, 0.0};
    const cf* xin = static_cast<const cf*>(a.in);
    const cf* cin = static_cast<const cf*>(ba.c_out);
    cf* gxo = static_cast<cf*>(a.out);
    // one wave of each SIMD per priority level: after a barrier, the LDS
    // serves the top wave of every SIMD first, which then starts its MFMAs
    // while the others still load, instead of all waves waiting together
    switch (wave >> 2) {
        case 0: __builtin_amdgcn_s_setprio(3); break;
        case 1: __builtin_amdgcn_s_setprio(2); break;
        case 2: __builtin_amdgcn_s_setprio(1); break;
        default: break;
    }
    if constexpr (D0) static_assert(LAY::kLogC == 0, "direct digit-0 I/O: digit 0 has stride 1");
    // D0: tile position of element 2q of this lane's digit-0 fibre, step it
    uint32_t dpos[NI];
#pragma unroll
    for (int it = 0; it < NI; ++it) {
        const DigitMap d = digit_map(fmap, 0);
        const uint32_t f = 256u * it | deposit8((uint32_t)wave, ~d.mask & 0xffu) | deposit8(lo, d.mask);
        dpos[it] = (f << 3) | (2u * hi);
    }

    // W (fragments fr) along digit J: src -> dst (in place when equal)
    auto pass = [&](auto J, const unsigned char* src, unsigned char* dst, const CFrag8& fr) {
        constexpr int j = decltype(J)::value;
        cpass8<NI>(src, dst, P0[j], P1[j], (uint32_t)logC + 3u * j, pad, fr);
    };
    // gradient sums of digit J (cotangent in Ct, activation act), then the
    // adjoint pass on Ct along J (skipped when ADJ is false); with RE, also
    // the pass of digit 0 from A into T1 (a_1 recomputed), whose operands
    // do not depend on the rest of the phase.  Every LDS load of the phase
    // is issued before the first MFMA, in the order of use, so the MFMAs of
    // the first step run while the later loads are still in flight.  The
    // adjoint pass rewrites only fibres this wave has just read.
    auto fused = [&](auto J, const unsigned char* act, auto ADJ, auto RE, auto OUT, int64_t origin) {
        constexpr int j = decltype(J)::value;
        constexpr bool adj = decltype(ADJ)::value != 0;
        constexpr bool re = decltype(RE)::value != 0;
        constexpr bool direct = decltype(OUT)::value != 0;  // D0, digit 0: result to gx
        static_assert(!direct || j == 0, "direct output: digit 0 only");
        const uint32_t h = (uint32_t)logC + 3u * j;
        float cv[NI][4], av[NI][4];
        cf x0[NI], x1[NI];
        PassRegs<NI> rr;
#pragma unroll
        for (int it = 0; it < NI; ++it) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t o = GB[j] + goff(j, 4 * it + u);
                cv[it][u] = *reinterpret_cast<const float*>(Cb + o);
                av[it][u] = *reinterpret_cast<const float*>(act + o);
            }
            if constexpr (adj) {
                const uint32_t so = lds_phys(digit_deposit(256u * it, h), pad) * 8u;
                x0[it] = *reinterpret_cast<const cf*>(Cb + P0[j] + so);
                x1[it] = *reinterpret_cast<const cf*>(Cb + P1[j] + so);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (re) cpass8_load<NI>(rr, Ab, P0[0], P1[0], (uint32_t)logC, pad);
        __builtin_amdgcn_sched_barrier(0);
        f32x4_c M = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int it = 0; it < NI; ++it) {
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (adj) {
                const uint32_t so = lds_phys(digit_deposit(256u * it, h), pad) * 8u;
                f32x4_c acc = {0.f, 0.f, 0.f, 0.f};
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(fh.a[0], x0[it].re, acc, 0, 0, 0);
                M = __builtin_amdgcn_mfma_f32_16x16x4f32(cv[it][0], av[it][0], M, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(fh.a[1], x0[it].im, acc, 0, 0, 0);
                M = __builtin_amdgcn_mfma_f32_16x16x4f32(cv[it][1], av[it][1], M, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(fh.a[2], x1[it].re, acc, 0, 0, 0);
                M = __builtin_amdgcn_mfma_f32_16x16x4f32(cv[it][2], av[it][2], M, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(fh.a[3], x1[it].im, acc, 0, 0, 0);
                M = __builtin_amdgcn_mfma_f32_16x16x4f32(cv[it][3], av[it][3], M, 0, 0, 0);
                if constexpr (direct) {
                    gstore16<nt_bwd_io<LAY>()>(gxo + origin + dpos[it],
                                               make_uint4(__float_as_uint(acc[0]), __float_as_uint(acc[1]),
                                                          __float_as_uint(acc[2]), __float_as_uint(acc[3])));
                } else {
                    *reinterpret_cast<cf*>(Cb + P0[j] + so) = cf{acc[0], acc[1]};
                    *reinterpret_cast<cf*>(Cb + P1[j] + so) = cf{acc[2], acc[3]};
                }
            } else {
#pragma unroll
                for (int u = 0; u < 4; ++u) M = __builtin_amdgcn_mfma_f32_16x16x4f32(cv[it][u], av[it][u], M, 0, 0, 0);
            }
        }
        if constexpr (re) cpass8_compute_store<NI>(rr, T1b, P0[0], P1[0], (uint32_t)logC, pad, fw);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int v = 0; v < 4; ++v) Md[v] += (double)M[v];
    };

    uint4 pa[NE], pc[NE];
    constexpr bool NT = nt_bwd_io<LAY>();
    TileWalk<NE, NT> tw;
    TileCursor cur = tw.init(a, tileE, pad);
    // the group input: tile layout, or (D0) the digit-0 pass layout
    auto fetch_a = [&](const TileCursor& c) {
        if constexpr (D0) {
#pragma unroll
            for (int it = 0; it < NI; ++it) pa[it] = gload16<NT>(xin + c.origin + dpos[it]);
        } else {
            tw.fetch(pa, xin, c);
        }
    };
    int64_t t = blockIdx.x;
    if (t < a.ntiles) {
        fetch_a(cur);
        tw.fetch(pc, cin, cur);
    }
    const bool want_gx = a.out != nullptr;
    [[maybe_unused]] f32x4_c a1keep[NI];  // D0: a_1 of the current tile (digit-0 pass layout)
    for (; t < a.ntiles; t += gridDim.x) {
#pragma unroll
        for (int j = 0; j < K; ++j) asm volatile("" : "+v"(P0[j]), "+v"(P1[j]), "+v"(GB[j]));
        if constexpr (D0) {
            // A into its slot and a_1 = W_0 A into T1, both from registers
            PassRegs<NI> r;
#pragma unroll
            for (int it = 0; it < NI; ++it) {
                cf v[2];
                *reinterpret_cast<uint4*>(v) = pa[it];
                r.x0[it] = v[0];
                r.x1[it] = v[1];
                const uint32_t so = lds_phys(256u * it << 3, pad) * 8u;
                *reinterpret_cast<cf*>(Ab + P0[0] + so) = v[0];
                *reinterpret_cast<cf*>(Ab + P1[0] + so) = v[1];
            }
            tw.commit(Cb, pc);
            cpass8_compute_store_keep<NI>(r, T1b, P0[0], P1[0], 0u, pad, fw, a1keep);
            __syncthreads();
        } else {
            tw.commit(Ab, pa);
            tw.commit(Cb, pc);
            __syncthreads();
        }
        const TileCursor nxt = tw.next(a, tileE, cur);
        if (t + gridDim.x < a.ntiles) {  // in flight while this tile is processed
            fetch_a(nxt);
            tw.fetch(pc, cin, nxt);
        }
        if constexpr (K >= 2 && !D0) {
            pass(IntC<0>{}, Ab, T1b, fw);  // a_1
            __syncthreads();
        }
        if constexpr (kPair) {
            cpass8<NI>(T1b, T2b, Q0[0], Q1[0], 3u, pad, fw);  // a_2
            wave_sync();
            cpass8<NI>(T2b, T1b, Q0[1], Q1[1], 6u, pad, fw);  // a_3 (replaces a_1)
            __syncthreads();
        } else if constexpr (K >= 3) {
            pass(IntC<1>{}, T1b, T2b, fw);  // a_2
            __syncthreads();
        }
        if constexpr (K == 4) {
            // a_3 replaces a_1 (recomputed from A once digit 3 is done); the
            // recompute shares the phase of digit 2, which reads only T2 and Ct
            if constexpr (!kPair) {
                pass(IntC<2>{}, T2b, T1b, fw);  // a_3
                __syncthreads();
            }
            fused(IntC<3>{}, T1b, IntC<1>{}, IntC<0>{}, IntC<0>{}, cur.origin);
            __syncthreads();
            if constexpr (D0) {
                // a_1 back into T1 from the registers of the first phase
                fused(IntC<2>{}, T2b, IntC<1>{}, IntC<0>{}, IntC<0>{}, cur.origin);
#pragma unroll
                for (int it = 0; it < NI; ++it) {
                    const uint32_t so = lds_phys(256u * it << 3, pad) * 8u;
                    *reinterpret_cast<cf*>(T1b + P0[0] + so) = cf{a1keep[it][0], a1keep[it][1]};
                    *reinterpret_cast<cf*>(T1b + P1[0] + so) = cf{a1keep[it][2], a1keep[it][3]};
                }
            } else {
                fused(IntC<2>{}, T2b, IntC<1>{}, IntC<1>{}, IntC<0>{}, cur.origin);  // and a_1 again
            }
            __syncthreads();
        }
        if constexpr (K == 3) {
            fused(IntC<2>{}, T2b, IntC<1>{}, IntC<0>{}, IntC<0>{}, cur.origin);
            __syncthreads();
        }
        if constexpr (K >= 2) {
            fused(IntC<1>{}, T1b, IntC<1>{}, IntC<0>{}, IntC<0>{}, cur.origin);
            if constexpr (kPair)
                wave_sync();
            else
                __syncthreads();
        }
        // out is null for the first digit group when only gW is wanted
        if (want_gx)
            fused(IntC<0>{}, Ab, IntC<1>{}, IntC<0>{}, IntC<D0 ? 1 : 0>{}, cur.origin);
        else
            fused(IntC<0>{}, Ab, IntC<0>{}, IntC<0>{}, IntC<0>{}, cur.origin);
        __syncthreads();
        if (want_gx && !D0) {
            tw.store(Cb, gxo, cur);
            __syncthreads();
        }
        cur = nxt;
    }
    // reduce the waves' 16 x 16 blocks in a fixed order, then form the
    // complex gradient (row / column m = 8 comp + e)
#pragma unroll
    for (int v = 0; v < 4; ++v) red[wave * 256 + (4 * (lane >> 4) + v) * 16 + (lane & 15)] = Md[v];
    __syncthreads();
    if (threadIdx.x < 64) {
        const int r = threadIdx.x >> 3, q = threadIdx.x & 7;
        auto Mv = [&](int mm, int nn) {
            double s = 0.0;
            for (int w = 0; w < kBwdThreads / 64; ++w) s += red[w * 256 + mm * 16 + nn];
            return s;
        };
        cd g;
        g.re = Mv(r, q) + Mv(8 + r, 8 + q);
        g.im = Mv(8 + r, q) - Mv(r, 8 + q);
        static_cast<cd*>(ba.partials)[(size_t)blockIdx.x * 64 + threadIdx.x] = g;
    }
}

}  // namespace gtt
