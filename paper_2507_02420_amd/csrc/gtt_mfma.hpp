// Digit-group pass on the matrix cores for radix 16 and 32.  Each digit pass
// is the product Y = W X (§3: Y = X W^T in the paper's row layout) with X the
// b x F matrix whose columns are the fibres of that digit, a dense
// contraction on 16 x 16 blocks of W:
//   A operand (W, 16 x 16 block): lane l holds W[i = l%16][4*(l/16) + 0..3];
//   B operand (X, 16 x 16 block): lane l holds X[4*(l/16) + 0..3][fibre l%16];
//   result: lane l holds Y[4*(l/16) + 0..3][fibre l%16].
// Input and output fragments have the same layout, so a wave reads four
// consecutive elements of its fibre from LDS, runs the MFMAs and writes four
// consecutive results back in place.  Radix 32 uses the 2 x 2 blocks of W.
//
// bf16 / f16 storage (16x16x16 MFMA): the tile stays in LDS in the storage
// type.  Every MFMA operand is the 16-bit rounding (nearest even) of the
// previous digit's FP32 result, so rounding each result once as it is
// written back is the same arithmetic as keeping it FP32 in LDS and
// rounding it on the next read, at half the LDS bytes per element (twice the
// elements per tile for the same LDS).  W is split into a high and a low
// 16-bit part (two MFMAs) so that its rounding adds no error; accumulation
// is FP32.
// FP32 storage (16x16x4 FP32 MFMA, see WFrag<float, B>): FP32 tile, W unsplit.
#pragma once

#include <type_traits>

#include "gtt_args.hpp"
#include "gtt_pass.hpp"
#include "gtt_types.hpp"

namespace gtt {

typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 h16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct MfmaOp;

template <>
struct MfmaOp<bf16> {
    using V = s16x4;
    using E = short;
    __device__ static V pack(const float (&x)[4]) {
        V r;
#pragma unroll
        for (int i = 0; i < 4; ++i) r[i] = __builtin_bit_cast(short, (__bf16)x[i]);
        return r;
    }
    __device__ static float unpack1(short v) { return __uint_as_float(((uint32_t)(uint16_t)v) << 16); }
    __device__ static void split(float w, short* hi, short* lo) {
        const __bf16 h = (__bf16)w;
        *hi = __builtin_bit_cast(short, h);
        *lo = __builtin_bit_cast(short, (__bf16)(w - (float)h));
    }
    __device__ static f32x4 mma(V a, V b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0); }
};

template <>
struct MfmaOp<f16> {
    using V = h16x4;
    using E = _Float16;
    __device__ static V pack(const float (&x)[4]) {
        V r;
#pragma unroll
        for (int i = 0; i < 4; ++i) r[i] = (_Float16)x[i];
        return r;
    }
    __device__ static void split(float w, _Float16* hi, _Float16* lo) {
        const _Float16 h = (_Float16)w;
        *hi = h;
        *lo = (_Float16)(w - (float)h);
    }
    __device__ static f32x4 mma(V a, V b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0); }
};

template <typename T, int B>
struct WFrag {
    static constexpr int NB = B / 16;
    typename MfmaOp<T>::V hi[NB][NB], lo[NB][NB];
};

// FP32 storage: W as FP32 operands of the 16x16x4 FP32 MFMA.  MFMA v of a
// 16 x 16 block contracts the columns 4q + v (q = lane / 16): lane (q, i)
// holds W[i][4q + v] and the fibre's element 4q + v, so the same fragment
// layout (four consecutive digit values per lane) takes four FP32 MFMAs
// instead of the 16-bit hi / lo pair.
template <int B>
struct WFrag<float, B> {
    static constexpr int NB = B / 16;
    float w[NB][NB][4];
};

template <typename T, int B>
__device__ __forceinline__ void load_w_frag16(WFrag<T, B>& wf, const float* __restrict__ Wg, int adjoint, int i,
                                              int q) {
    using Op = MfmaOp<T>;
#pragma unroll
    for (int bi = 0; bi < WFrag<T, B>::NB; ++bi)
#pragma unroll
        for (int bk = 0; bk < WFrag<T, B>::NB; ++bk)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = 16 * bi + i, c = 16 * bk + 4 * q + v;
                const float w = adjoint ? Wg[c * B + r] : Wg[r * B + c];
                typename Op::E h, l;
                Op::split(w, &h, &l);
                wf.hi[bi][bk][v] = h;
                wf.lo[bi][bk][v] = l;
            }
}

template <typename T, int B>
__device__ __forceinline__ void load_w_frag(WFrag<T, B>& wf, const PassArgs& a) {
    const float* __restrict__ Wg = static_cast<const float*>(a.W);
    const int lane = threadIdx.x & 63;
    const int i = lane & 15, q = lane >> 4;
    if constexpr (std::is_same<T, float>::value) {
#pragma unroll
        for (int bi = 0; bi < WFrag<T, B>::NB; ++bi)
#pragma unroll
            for (int bk = 0; bk < WFrag<T, B>::NB; ++bk)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = 16 * bi + i, c = 16 * bk + 4 * q + v;
                    wf.w[bi][bk][v] = a.adjoint ? Wg[c * B + r] : Wg[r * B + c];
                }
        return;
    } else {
        load_w_frag16<T, B>(wf, Wg, a.adjoint, i, q);
    }
}

// W (fragments wf) along digit j of every fibre of an FP32 tile on the FP32
// MFMA: src -> dst (in place when equal: each lane reads its fibres' values
// before it writes them).  NT threads per work-group.
template <int B, int NT = kThreads>
__device__ __forceinline__ void mfma_pass_f32(const float* src, float* dst, const PassArgs& a, int j, uint32_t rows,
                                              const WFrag<float, B>& wf) {
    constexpr int NB = B / 16;
    const uint32_t F = (rows << a.logC) / B;
    const uint32_t step = (uint32_t)a.bpow[j] << a.logC;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int q = lane >> 4;
    const uint32_t ngrp = (F + 15) / 16;
    const int pad = a.pad_shift;
    // element (16 h + 4 q + v) of a fibre sits at lam0 | that * step, with
    // the digit's bits zero in lam0: lds_phys splits into a per-fibre base,
    // a per-lane part (q) and a uniform part (h, v)
    const uint32_t qoff = lds_phys(4u * q * step, pad);
    uint32_t off[NB][4];
#pragma unroll
    for (int h = 0; h < NB; ++h)
#pragma unroll
        for (int v = 0; v < 4; ++v) off[h][v] = lds_phys((16u * h + v) * step, pad);
    // The fibre's position is f with LB zero bits (digit j) inserted at bit
    // hj = logC + LB j; for f = 16 grp + i (disjoint bits) the insertion and
    // lds_phys are additive, so the lane part is fixed for the stage and the
    // group part is work-group uniform.
    constexpr uint32_t LB = B == 16 ? 4u : 5u;
    const uint32_t hj = (uint32_t)a.logC + LB * (uint32_t)j;
    auto ins = [&](uint32_t v) { return ((v >> hj) << (hj + LB)) | (v & ((1u << hj) - 1u)); };
    const uint32_t lane_base = lds_phys(ins((uint32_t)(lane & 15)), pad) + qoff;
    for (uint32_t grp = wave; grp < ngrp; grp += NT / 64) {
        const uint32_t f = grp * 16 + (lane & 15);
        const bool valid = f < F;
        const uint32_t base = lds_phys(ins(__builtin_amdgcn_readfirstlane(grp) * 16u), pad) + lane_base;
        float x[NB][4];
#pragma unroll
        for (int h = 0; h < NB; ++h)
#pragma unroll
            for (int v = 0; v < 4; ++v) x[h][v] = valid ? src[base + off[h][v]] : 0.f;
        f32x4 acc[NB];
#pragma unroll
        for (int bi = 0; bi < NB; ++bi) {
            acc[bi] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int bk = 0; bk < NB; ++bk)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    acc[bi] = __builtin_amdgcn_mfma_f32_16x16x4f32(wf.w[bi][bk][v], x[bk][v], acc[bi], 0, 0, 0);
        }
        if (valid) {
#pragma unroll
            for (int bi = 0; bi < NB; ++bi)
#pragma unroll
                for (int v = 0; v < 4; ++v) dst[base + off[bi][v]] = acc[bi][v];
        }
    }
}

// W along digit j of every fibre of the FP32 tile, in place, on the FP32 MFMA.
template <typename T, int B>
__device__ __forceinline__ void mfma_stage(float* lds, const PassArgs& a, int j, uint32_t rows,
                                           const WFrag<T, B>& wf) {
    static_assert(std::is_same<T, float>::value, "16-bit storage runs mfma_stage16");
    mfma_pass_f32<B>(lds, lds, a, j, rows, wf);
}

// Weight-gradient sums of digit j over the fibres of an FP32 tile on the
// FP32 MFMA: M[r][q] = sum over fibres f of c_f[r] a_f[q] (real data: the
// rank-1 terms c a^T).  With K = four fibres per MFMA, lane (k = lane / 16,
// m = lane % 16) supplies element m (of each 16-row block) of fibre
// 4 grp + k of both tiles: the A operand c[m] (rows) and the B operand a[m]
// (columns).  The FP32 chain covers one digit of one tile (the fibres a wave
// takes, four per step) and is then added into the FP64 accumulators Md:
// lane (q, i), value v holds block (bi, bj) entry (16 bi + 4 q + v, 16 bj + i).
template <int B, int NT = kThreads>
__device__ __forceinline__ void mfma_gw_f32(const float* ct, const float* at, const PassArgs& a, int j,
                                            uint32_t rows, double (&Md)[B / 16][B / 16][4]) {
    constexpr int NB = B / 16;
    const uint32_t F = (rows << a.logC) / B;
    const uint32_t step = (uint32_t)a.bpow[j] << a.logC;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const uint32_t m = (uint32_t)(lane & 15), k = (uint32_t)(lane >> 4);
    const int pad = a.pad_shift;
    constexpr uint32_t LB = B == 16 ? 4u : 5u;
    const uint32_t hj = (uint32_t)a.logC + LB * (uint32_t)j;
    auto ins = [&](uint32_t v) { return ((v >> hj) << (hj + LB)) | (v & ((1u << hj) - 1u)); };
    // fibre 4 grp + k (disjoint bits) and element 16 bi + m: every part of
    // the position is additive under lds_phys
    uint32_t eoff[NB];
#pragma unroll
    for (int bi = 0; bi < NB; ++bi) eoff[bi] = lds_phys((16u * bi + m) * step, pad);
    const uint32_t kbase = lds_phys(ins(k), pad);
    const uint32_t ngrp = (F + 3) / 4;
    f32x4 M[NB][NB];
#pragma unroll
    for (int bi = 0; bi < NB; ++bi)
#pragma unroll
        for (int bj = 0; bj < NB; ++bj) M[bi][bj] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (uint32_t grp = wave; grp < ngrp; grp += NT / 64) {
        const bool valid = grp * 4 + k < F;
        const uint32_t base = lds_phys(ins(__builtin_amdgcn_readfirstlane(grp) * 4u), pad) + kbase;
        float cv[NB], av[NB];
#pragma unroll
        for (int bi = 0; bi < NB; ++bi) {
            cv[bi] = valid ? ct[base + eoff[bi]] : 0.f;
            av[bi] = valid ? at[base + eoff[bi]] : 0.f;
        }
#pragma unroll
        for (int bi = 0; bi < NB; ++bi)
#pragma unroll
            for (int bj = 0; bj < NB; ++bj)
                M[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x4f32(cv[bi], av[bj], M[bi][bj], 0, 0, 0);
    }
#pragma unroll
    for (int bi = 0; bi < NB; ++bi)
#pragma unroll
        for (int bj = 0; bj < NB; ++bj)
#pragma unroll
            for (int v = 0; v < 4; ++v) Md[bi][bj][v] += (double)M[bi][bj][v];
}

// ---- 16-bit tiles ----------------------------------------------------------
// Element x of a 16-bit tile sits at 16-bit position
// 2 * lds_phys(x >> 1, pad) + (x & 1): the pads count 32-bit words, so an
// aligned element pair is one word and a 16-byte vector (eight elements)
// four consecutive words (pad shifts >= 2).  Like lds_phys, the map is
// additive over disjoint bits.
__device__ __forceinline__ uint32_t lds_phys16(uint32_t x, int pad) { return 2u * lds_phys(x >> 1, pad) + (x & 1u); }

template <typename T>
__device__ __forceinline__ void tile_load16(uint16_t* lds, const PassArgs& a, const T* __restrict__ in, int64_t t,
                                            uint32_t rows) {
    static_assert(sizeof(T) == 2, "16-bit storage");
    const uint32_t tileE = rows << a.logC;
    const bool contig = a.mode == kContigVec || a.mode == kContigScalar;
    const int64_t hb = contig ? 0 : tile_hb(a, t);
    const int64_t l = contig ? 0 : t - hb * a.L;
    const uint16_t* __restrict__ src = reinterpret_cast<const uint16_t*>(in);
    uint32_t* w = reinterpret_cast<uint32_t*>(lds);
    if (a.mode == kContigVec || a.mode == kRowVec) {
        const uint32_t nvec = tileE / 8;
        for (uint32_t i0 = 0; i0 < nvec; i0 += kLoadBatch * kThreads) {
            uint4 buf[kLoadBatch];
#pragma unroll
            for (int v = 0; v < kLoadBatch; ++v) {
                const uint32_t i = i0 + threadIdx.x + v * kThreads;
                if (i < nvec) buf[v] = *reinterpret_cast<const uint4*>(src + vec_offset<T>(a, t, i, hb, l, tileE));
            }
#pragma unroll
            for (int v = 0; v < kLoadBatch; ++v) {
                const uint32_t i = i0 + threadIdx.x + v * kThreads;
                if (i < nvec) {
                    uint32_t d[4] = {buf[v].x, buf[v].y, buf[v].z, buf[v].w};
                    if (a.cut >= 0) {  // natural-order mask of the filter
                        const int64_t off = vec_offset<T>(a, t, i, hb, l, tileE);
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            const bool low = (off + e) % a.N < a.cut;
                            if (low == (a.cut_keep_high != 0)) d[e >> 1] &= (e & 1) ? 0x0000ffffu : 0xffff0000u;
                        }
                    }
                    const uint32_t ph = lds_phys(4u * i, a.pad_shift);
#pragma unroll
                    for (int e = 0; e < 4; ++e) w[ph + e] = d[e];
                }
            }
        }
    } else {
        for (uint32_t i0 = 0; i0 < tileE; i0 += kLoadBatch * kThreads) {
            uint16_t buf[kLoadBatch];
#pragma unroll
            for (int v = 0; v < kLoadBatch; ++v) {
                const uint32_t i = i0 + threadIdx.x + v * kThreads;
                if (i < tileE) {
                    const int64_t off = elem_offset(a, t, i, hb, l, tileE);
                    if (off >= 0 && (a.cut < 0 || ((off % a.N < a.cut) != (a.cut_keep_high != 0))))
                        buf[v] = src[off];
                    else
                        buf[v] = 0;
                }
            }
#pragma unroll
            for (int v = 0; v < kLoadBatch; ++v) {
                const uint32_t i = i0 + threadIdx.x + v * kThreads;
                if (i < tileE) lds[lds_phys16(i, a.pad_shift)] = buf[v];
            }
        }
    }
}

template <typename T>
__device__ __forceinline__ void tile_store16(const uint16_t* lds, const PassArgs& a, T* __restrict__ out, int64_t t,
                                             uint32_t rows) {
    static_assert(sizeof(T) == 2, "16-bit storage");
    const uint32_t tileE = rows << a.logC;
    const bool contig = a.mode == kContigVec || a.mode == kContigScalar;
    const int64_t hb = contig ? 0 : tile_hb(a, t);
    const int64_t l = contig ? 0 : t - hb * a.L;
    uint16_t* __restrict__ dst = reinterpret_cast<uint16_t*>(out);
    const uint32_t* w = reinterpret_cast<const uint32_t*>(lds);
    if (a.mode == kContigVec || a.mode == kRowVec) {
        const uint32_t nvec = tileE / 8;
        for (uint32_t i = threadIdx.x; i < nvec; i += kThreads) {
            const uint32_t ph = lds_phys(4u * i, a.pad_shift);
            const uint4 d = make_uint4(w[ph], w[ph + 1], w[ph + 2], w[ph + 3]);
            gstore16<true>(dst + vec_offset<T>(a, t, i, hb, l, tileE), d);
        }
    } else {
        for (uint32_t i = threadIdx.x; i < tileE; i += kThreads) {
            const int64_t off = elem_offset(a, t, i, hb, l, tileE);
            if (off >= 0) dst[off] = lds[lds_phys16(i, a.pad_shift)];
        }
    }
}

// W along digit j of every fibre of a 16-bit tile, in place: the values
// read are the MFMA operands as they stand, the FP32 results are rounded to
// the storage type as they are written back.  A contiguous digit (step 1)
// moves the four elements of a fragment as two 32-bit words.
template <typename T, int B>
__device__ __forceinline__ void mfma_stage16(uint16_t* lds, const PassArgs& a, int j, uint32_t rows,
                                             const WFrag<T, B>& wf) {
    using Op = MfmaOp<T>;
    using V = typename Op::V;
    constexpr int NB = B / 16;
    const uint32_t F = (rows << a.logC) / B;
    const uint32_t step = (uint32_t)a.bpow[j] << a.logC;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int q = lane >> 4;
    const uint32_t ngrp = (F + 15) / 16;
    const int pad = a.pad_shift;
    const uint32_t qoff = lds_phys16(4u * q * step, pad);
    uint32_t off[NB][4];
#pragma unroll
    for (int h = 0; h < NB; ++h)
#pragma unroll
        for (int v = 0; v < 4; ++v) off[h][v] = lds_phys16((16u * h + v) * step, pad);
    constexpr uint32_t LB = B == 16 ? 4u : 5u;
    const uint32_t hj = (uint32_t)a.logC + LB * (uint32_t)j;
    auto ins = [&](uint32_t v) { return ((v >> hj) << (hj + LB)) | (v & ((1u << hj) - 1u)); };
    const uint32_t lane_base = lds_phys16(ins((uint32_t)(lane & 15)), pad) + qoff;
    // step 1: every fragment starts at an even position (all address terms
    // are even), so elements (0, 1) and (2, 3) are words
    const bool pairs = step == 1u;
    uint32_t* w32 = reinterpret_cast<uint32_t*>(lds);
    for (uint32_t grp = wave; grp < ngrp; grp += kThreads / 64) {
        const uint32_t f = grp * 16 + (lane & 15);
        const bool valid = f < F;
        const uint32_t base = lds_phys16(ins(__builtin_amdgcn_readfirstlane(grp) * 16u), pad) + lane_base;
        V xb[NB];
#pragma unroll
        for (int h = 0; h < NB; ++h) {
            uint32_t d0 = 0, d1 = 0;
            if (valid) {
                if (pairs) {
                    d0 = w32[(base + off[h][0]) >> 1];
                    d1 = w32[(base + off[h][2]) >> 1];
                } else {
                    d0 = (uint32_t)lds[base + off[h][0]] | ((uint32_t)lds[base + off[h][1]] << 16);
                    d1 = (uint32_t)lds[base + off[h][2]] | ((uint32_t)lds[base + off[h][3]] << 16);
                }
            }
            xb[h] = __builtin_bit_cast(V, make_uint2(d0, d1));
        }
        f32x4 acc[NB];
#pragma unroll
        for (int bi = 0; bi < NB; ++bi) {
            acc[bi] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int bk = 0; bk < NB; ++bk) {
                acc[bi] = Op::mma(wf.hi[bi][bk], xb[bk], acc[bi]);
                acc[bi] = Op::mma(wf.lo[bi][bk], xb[bk], acc[bi]);
            }
        }
        if (valid) {
#pragma unroll
            for (int bi = 0; bi < NB; ++bi) {
                const float r[4] = {acc[bi][0], acc[bi][1], acc[bi][2], acc[bi][3]};
                const uint2 d = __builtin_bit_cast(uint2, Op::pack(r));
                if (pairs) {
                    w32[(base + off[bi][0]) >> 1] = d.x;
                    w32[(base + off[bi][2]) >> 1] = d.y;
                } else {
                    lds[base + off[bi][0]] = (uint16_t)d.x;
                    lds[base + off[bi][1]] = (uint16_t)(d.x >> 16);
                    lds[base + off[bi][2]] = (uint16_t)d.y;
                    lds[base + off[bi][3]] = (uint16_t)(d.y >> 16);
                }
            }
        }
    }
}

template <typename T, int B>
__global__ __launch_bounds__(kThreads) void gtt_pass_mfma_kernel(PassArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    WFrag<T, B> wf;
    load_w_frag<T, B>(wf, a);
    if constexpr (std::is_same<T, float>::value) {
        // persistent grid, next tile prefetched into registers (tile_loop)
        float* lds = reinterpret_cast<float*>(smem_raw);
        tile_loop<T, float, true>(lds, a, [&](float* t, uint32_t rows, int64_t) {
            for (int j = 0; j < a.k; ++j) {
                mfma_stage<T, B>(t, a, j, rows, wf);
                __syncthreads();
            }
            return false;
        });
    } else {
        // The work-groups loop over tiles (the launch is as large as the
        // device holds at once).  Vector tiles of up to 16384 elements have
        // the next tile's loads in flight into 32 registers per thread while
        // the current one runs its digits: occupancy is set by LDS here, and
        // those registers fit under its limit.
        uint16_t* lds = reinterpret_cast<uint16_t*>(smem_raw);
        const uint32_t rows = (uint32_t)a.P * (uint32_t)a.G;
        const uint32_t tileE = rows << a.logC;
        const T* in = static_cast<const T*>(a.in);
        T* out = static_cast<T*>(a.out);
        const bool vec = a.mode == kContigVec || a.mode == kRowVec;
        const bool pf = vec && a.cut < 0 && (int64_t)gridDim.x < a.ntiles && tileE / 8 <= (uint32_t)(kPfVec * kThreads);
        uint4 r[kPfVec];
        // offsets recomputed per tile behind an opaque thread index, so that
        // they do not stay live in registers across the loop
        auto fetch = [&](int64_t t) {
            const bool contig = a.mode == kContigVec;
            const int64_t hb = contig ? 0 : tile_hb(a, t);
            const int64_t l = contig ? 0 : t - hb * a.L;
            uint32_t tid = threadIdx.x;
            asm volatile("" : "+v"(tid));
            // every register written (zero past the tile), so that the old
            // contents are dead here
#pragma unroll
            for (int v = 0; v < kPfVec; ++v) {
                const uint32_t i = tid + v * kThreads;
                uint4 q = make_uint4(0u, 0u, 0u, 0u);
                if (i < tileE / 8) q = gload16<true>(in + vec_offset<T>(a, t, i, hb, l, tileE));
                r[v] = q;
            }
        };
        auto commit = [&]() {
            uint32_t tid = threadIdx.x;
            asm volatile("" : "+v"(tid));
            uint32_t* w = reinterpret_cast<uint32_t*>(lds);
#pragma unroll
            for (int v = 0; v < kPfVec; ++v) {
                const uint32_t i = tid + v * kThreads;
                if (i < tileE / 8) {
                    const uint32_t ph = lds_phys(4u * i, a.pad_shift);
                    w[ph] = r[v].x;
                    w[ph + 1] = r[v].y;
                    w[ph + 2] = r[v].z;
                    w[ph + 3] = r[v].w;
                }
            }
        };
        int64_t t = blockIdx.x;
        if (pf && t < a.ntiles) fetch(t);
        for (; t < a.ntiles; t += gridDim.x) {
            if (pf)
                commit();
            else
                tile_load16<T>(lds, a, in, t, rows);
            __syncthreads();
            if (pf && t + gridDim.x < a.ntiles) fetch(t + gridDim.x);
            for (int j = 0; j < a.k; ++j) {
                mfma_stage16<T, B>(lds, a, j, rows, wf);
                __syncthreads();
            }
            tile_store16<T>(lds, a, out, t, rows);
            __syncthreads();
        }
    }
}

}  // namespace gtt
