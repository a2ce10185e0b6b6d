// Fused digit-group pass: one HBM round trip applies W along k consecutive
// base-b digits (§3: each level of the fast algorithm is the product
// Y = X W^T along one digit; the levels act on different tensor factors of
// Def. 2.4 and therefore commute, so any k of them can be done on one tile).
//
// A work-group owns one tile (P hi blocks x G = b^k group positions x C lo
// columns, see gtt_args.hpp).  It
//   1. streams the tile from HBM into LDS with coalesced accesses
//      (16-byte vectors where the layout allows), converting storage to the
//      compute dtype;
//   2. runs the k digits as ceil(k / RD) register super-stages: each thread
//      gathers a B^RD block spanning RD digits from LDS, applies W along those
//      RD digits in registers and scatters the block back;
//   3. streams the tile back to HBM.
// Every tile is read completely before it is written, and tiles are disjoint
// sets of positions that map onto themselves, so in-place (in == out) is safe.
#pragma once

#include <type_traits>

#include "gtt_args.hpp"
#include "gtt_types.hpp"

namespace gtt {

__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv& f) {
    return (__umulhi(n, f.m) + n) >> f.s;
}

// hi block of tile t (t = hb * L + l, the tile's column block l < L): one
// multiply-high while t and L are below 2^31, a 64-bit division beyond
__device__ __forceinline__ int64_t tile_hb(const PassArgs& a, int64_t t) {
    if (a.L == 1) return t;
    if (t < 0x80000000LL && a.L < 0x80000000LL) return (int64_t)fdiv((uint32_t)t, a.divL);
    return t / a.L;
}

template <int B, int R>
struct IPow {
    static constexpr int value = B * IPow<B, R - 1>::value;
};
template <int B>
struct IPow<B, 0> {
    static constexpr int value = 1;
};

// register digits per super-stage: blocks of at most 16 elements
template <int B>
struct RegDigits {
    static constexpr int v = (B == 2) ? 4 : (B == 3 || B == 4) ? 2 : 1;
};

// ---------------------------------------------------------------------------
// W along digit D of a register block of B^R values (digit 0 = stride 1).
// ---------------------------------------------------------------------------
template <typename C, int B, int R, int D>
__device__ __forceinline__ void block_digit(C (&v)[(IPow<B, R>::value)], const C (&w)[B * B]) {
    constexpr int st = IPow<B, D>::value;
    constexpr int n = IPow<B, R>::value;
#pragma unroll
    for (int base = 0; base < n; ++base) {
        if ((base / st) % B != 0) continue;  // base must have digit D == 0
        C in[B];
#pragma unroll
        for (int q = 0; q < B; ++q) in[q] = v[base + q * st];
#pragma unroll
        for (int r = 0; r < B; ++r) {
            C acc = cmul(w[r * B], in[0]);
#pragma unroll
            for (int q = 1; q < B; ++q) acc = cmac(acc, w[r * B + q], in[q]);
            v[base + r * st] = acc;
        }
    }
}

// W^H along digit D of a register block: v[r] <- sum_q conj(W[q][r]) v[q]
// (the adjoint taken from W's registers: no second matrix)
template <typename C, int B, int R, int D>
__device__ __forceinline__ void block_digit_adj(C (&v)[(IPow<B, R>::value)], const C (&w)[B * B]) {
    constexpr int st = IPow<B, D>::value;
    constexpr int n = IPow<B, R>::value;
#pragma unroll
    for (int base = 0; base < n; ++base) {
        if ((base / st) % B != 0) continue;  // base must have digit D == 0
        C in[B];
#pragma unroll
        for (int q = 0; q < B; ++q) in[q] = v[base + q * st];
#pragma unroll
        for (int r = 0; r < B; ++r) {
            C acc = cmac_conj(czero<C>(), in[0], w[r]);
#pragma unroll
            for (int q = 1; q < B; ++q) acc = cmac_conj(acc, in[q], w[q * B + r]);
            v[base + r * st] = acc;
        }
    }
}

// The same for the integer radix-2 Hadamard W = [[1, 1], [1, -1]]: one add
// and one subtract per pair (wrap-around arithmetic, so the result is the
// same as with the multiplies, which are quarter-rate for 32-bit integers).
template <typename C, int R, int D>
__device__ __forceinline__ void block_digit_h2(C (&v)[(IPow<2, R>::value)]) {
    constexpr int st = IPow<2, D>::value;
    constexpr int n = IPow<2, R>::value;
#pragma unroll
    for (int base = 0; base < n; ++base) {
        if ((base / st) % 2 != 0) continue;
        const C x0 = v[base], x1 = v[base + st];
        v[base] = x0 + x1;
        v[base + st] = x0 - x1;
    }
}
template <typename C, int R, int D>
struct BlockAllH2 {
    __device__ __forceinline__ static void run(C (&v)[(IPow<2, R>::value)]) {
        block_digit_h2<C, R, D>(v);
        BlockAllH2<C, R, D + 1>::run(v);
    }
};
template <typename C, int R>
struct BlockAllH2<C, R, R> {
    __device__ __forceinline__ static void run(C (&)[(IPow<2, R>::value)]) {}
};

template <typename C, int B, int R, int D>
struct BlockAll {
    __device__ __forceinline__ static void run(C (&v)[(IPow<B, R>::value)], const C (&w)[B * B]) {
        block_digit<C, B, R, D>(v, w);
        BlockAll<C, B, R, D + 1>::run(v, w);
    }
};
template <typename C, int B, int R>
struct BlockAll<C, B, R, R> {
    __device__ __forceinline__ static void run(C (&)[(IPow<B, R>::value)], const C (&)[B * B]) {}
};

// pad_shift of an unpadded tile (all three shifts 31)
constexpr int kPadNone = 31 | (31 << 8) | (31 << 16);

// LDS position of tile element lam.  pad_shift packs three shift amounts
// (bits 0-7, 8-15, 16-23; 31 = none): one pad element after every 2^p1, 2^p2
// and 2^p3 elements.  With p1, p2, p3 one digit apart, every power-of-b
// stride of a digit fibre becomes an odd number of banks, so the lanes of a
// wave that walk a fibre hit distinct banks.
__device__ __forceinline__ uint32_t lds_phys(uint32_t lam, int pad_shift) {
    return lam + (lam >> (pad_shift & 31)) + (lam >> ((pad_shift >> 8) & 31)) + (lam >> ((pad_shift >> 16) & 31));
}

// LDS elements of a tile of tileE elements under lds_phys
__device__ __forceinline__ uint32_t lds_tile_elems(uint32_t tileE, int pad_shift) {
    return tileE + (tileE >> (pad_shift & 31)) + (tileE >> ((pad_shift >> 8) & 31)) +
           (tileE >> ((pad_shift >> 16) & 31)) + 1u;
}

// One super-stage: digits j .. j+R-1 of the group, all fibres of the tile.
// For a power-of-two radix the block's positions lam0 | m * step have the
// register digits in bits where lam0 is zero, and lds_phys is additive over
// numbers with disjoint bits, so every position costs one add of a
// work-group-uniform offset; without padding positions are linear.
//
// GOUT: the group's last super-stage writes its results straight to global
// memory at gout instead of back to LDS (contiguous tiles, or row tiles of
// one hi block; gt0 = the tile's first global element).  Lanes with
// consecutive fibres hold consecutive tile positions, so each store of a
// wave covers whole runs of contiguous elements.
template <typename C, int B, int R, bool GOUT = false>
__device__ __forceinline__ void super_stage(C* lds, const PassArgs& a, int j, uint32_t rows,
                                           const C (&w)[B * B], bool h2 = false, C* gout = nullptr,
                                           int64_t gt0 = 0) {
    constexpr int NB = IPow<B, R>::value;
    constexpr bool kPow2 = (B & (B - 1)) == 0;
    const uint32_t Cm = (1u << a.logC) - 1u;
    const uint32_t F = (rows << a.logC) / NB;
    const uint32_t bj = (uint32_t)a.bpow[j];
    const uint32_t bjr = (uint32_t)a.bpow[j + R];
    const uint32_t step = bj << a.logC;
    const int pad = a.pad_shift;
    const bool linear = pad == kPadNone;
    uint32_t off[NB];
#pragma unroll
    for (int m = 0; m < NB; ++m) off[m] = (kPow2 && !linear) ? lds_phys(m * step, pad) : m * step;
    for (uint32_t f = threadIdx.x; f < F; f += kThreads) {
        const uint32_t c = f & Cm;
        const uint32_t f1 = f >> a.logC;
        const uint32_t Q = fdiv(f1, a.divb[j]);
        const uint32_t glo = f1 - Q * bj;
        const uint32_t lam0 = ((Q * bjr + glo) << a.logC) | c;
        uint32_t idx[NB];
        if (kPow2 || linear) {
            const uint32_t ph0 = linear ? lam0 : lds_phys(lam0, pad);
#pragma unroll
            for (int m = 0; m < NB; ++m) idx[m] = ph0 + off[m];
        } else {
#pragma unroll
            for (int m = 0; m < NB; ++m) idx[m] = lds_phys(lam0 + m * step, pad);
        }
        C v[NB];
#pragma unroll
        for (int m = 0; m < NB; ++m) v[m] = lds[idx[m]];
        if constexpr (B == 2 && std::is_same<C, uint32_t>::value) {
            if (h2)  // work-group uniform
                BlockAllH2<C, R, 0>::run(v);
            else
                BlockAll<C, B, R, 0>::run(v, w);
        } else {
            BlockAll<C, B, R, 0>::run(v, w);
        }
        if constexpr (GOUT) {
            // position lam0 + m * step: element lam0 + m * step of a
            // contiguous tile, row (lam0 >> logC) + m * b^j of a row tile
            // (byte offsets from the tile's base fit 32 bits: checked by the caller)
            const bool row = a.mode == kRowVec;
            const uint32_t S32 = (uint32_t)a.S;
            const uint32_t o0 = row ? (lam0 >> a.logC) * S32 + (lam0 & Cm) : lam0;
            const uint32_t om = row ? bj * S32 : step;
            char* gb = reinterpret_cast<char*>(gout + gt0);
#pragma unroll
            for (int m = 0; m < NB; ++m)
                *reinterpret_cast<C*>(gb + (uint32_t)((o0 + (uint32_t)m * om) * (uint32_t)sizeof(C))) = v[m];
        } else {
#pragma unroll
            for (int m = 0; m < NB; ++m) lds[idx[m]] = v[m];
        }
    }
}

// With gout, the last super-stage stores to global memory (see super_stage)
// and no barrier follows it: the caller's barrier after the tile orders its
// LDS reads before the next tile's LDS writes.
template <typename C, int B, int RD>
__device__ __forceinline__ void run_stages(C* lds, const PassArgs& a, uint32_t rows, const C (&w)[B * B],
                                           bool h2 = false, C* gout = nullptr, int64_t gt0 = 0) {
    for (int j = 0; j < a.k; j += RD) {
        const int r = (a.k - j) < RD ? (a.k - j) : RD;
        if (gout && j + r == a.k) {
            if constexpr (RD >= 4) {
                if (r == 4) { super_stage<C, B, 4, true>(lds, a, j, rows, w, h2, gout, gt0); return; }
            }
            if constexpr (RD >= 3) {
                if (r == 3) { super_stage<C, B, 3, true>(lds, a, j, rows, w, h2, gout, gt0); return; }
            }
            if constexpr (RD >= 2) {
                if (r == 2) { super_stage<C, B, 2, true>(lds, a, j, rows, w, h2, gout, gt0); return; }
            }
            super_stage<C, B, 1, true>(lds, a, j, rows, w, h2, gout, gt0);
            return;
        }
        if constexpr (RD >= 4) {
            if (r == 4) { super_stage<C, B, 4>(lds, a, j, rows, w, h2); __syncthreads(); continue; }
        }
        if constexpr (RD >= 3) {
            if (r == 3) { super_stage<C, B, 3>(lds, a, j, rows, w, h2); __syncthreads(); continue; }
        }
        if constexpr (RD >= 2) {
            if (r == 2) { super_stage<C, B, 2>(lds, a, j, rows, w, h2); __syncthreads(); continue; }
        }
        super_stage<C, B, 1>(lds, a, j, rows, w, h2);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Tile <-> LDS movement
// ---------------------------------------------------------------------------
template <typename T>
struct Vec16 {
    static constexpr int V = 16 / sizeof(T);  // storage elements per 16 bytes
};

// global offset (elements) of the start of row r of the tile
__device__ __forceinline__ int64_t row_offset(const PassArgs& a, int64_t hb, int64_t l, uint32_t r) {
    const uint32_t p = (a.P == 1) ? 0u : fdiv(r, a.divG);
    const uint32_t g = r - p * (uint32_t)a.G;
    return (hb * a.P + p) * ((int64_t)a.G * a.S) + (int64_t)g * a.S + (l << a.logC);
}

// All global loads of a thread are issued before the first LDS write, so a
// thread has up to kLoadBatch accesses in flight instead of one.
constexpr int kLoadBatch = 8;

// global element offset of 16-byte vector i of tile t (vector modes)
template <typename T>
__device__ __forceinline__ int64_t vec_offset(const PassArgs& a, int64_t t, uint32_t i, int64_t hb, int64_t l,
                                              uint32_t tileE) {
    constexpr int V = Vec16<T>::V;
    if (a.mode == kContigVec) return t * (int64_t)tileE + (int64_t)i * V;
    const int lcv = a.logC - __builtin_ctz(V);  // log2(vectors per row)
    const uint32_t r = i >> lcv;
    const uint32_t cc = i & ((1u << lcv) - 1u);
    return row_offset(a, hb, l, r) + (int64_t)cc * V;
}

// global element offset of element i of tile t (scalar modes); -1 when the
// element lies past the last valid column of a partial column block
__device__ __forceinline__ int64_t elem_offset(const PassArgs& a, int64_t t, uint32_t i, int64_t hb, int64_t l,
                                               uint32_t tileE) {
    if (a.mode == kContigScalar) return t * (int64_t)tileE + i;
    const uint32_t r = i >> a.logC;
    const uint32_t c = i & ((1u << a.logC) - 1u);
    if ((int64_t)c >= a.S - (l << a.logC)) return -1;
    return row_offset(a, hb, l, r) + c;
}

// Vector-mode addresses of a tile as a walk: vector i = tid + m * kThreads
// of tile t lies at global element g0 + m * gstep and at LDS element
// l0 + m * lstep.  This holds for contiguous tiles, and for row tiles of one
// hi block (P == 1) whose rows have at most kThreads vectors; on the LDS
// side lds_phys is additive over the step when every pad period divides
// kThreads * V (vec_walk_ok checks both).
struct VecWalk {
    int64_t g0, gstep;
    uint32_t l0, lstep;
};
template <typename T>
__device__ __forceinline__ bool vec_walk_ok(const PassArgs& a) {
    constexpr int lv = __builtin_ctz(Vec16<T>::V);
    constexpr int lim = __builtin_ctz(kThreads) + lv;
    for (int k = 0; k < 3; ++k) {
        const int sh = (a.pad_shift >> (8 * k)) & 31;
        if (sh != 31 && sh > lim) return false;
    }
    if (a.mode == kContigVec) return true;
    return a.mode == kRowVec && a.P == 1 && a.logC >= lv && a.logC - lv <= __builtin_ctz(kThreads);
}
template <typename T>
__device__ __forceinline__ VecWalk vec_walk(const PassArgs& a, int64_t t, uint32_t tid, uint32_t tileE) {
    constexpr int V = Vec16<T>::V;
    VecWalk w;
    if (a.mode == kContigVec) {
        w.g0 = t * (int64_t)tileE + (int64_t)tid * V;
        w.gstep = (int64_t)kThreads * V;
    } else {
        const int lcv = a.logC - __builtin_ctz(V);
        const int64_t hb = tile_hb(a, t);
        const int64_t l = t - hb * a.L;
        w.g0 = hb * ((int64_t)a.G * a.S) + (l << a.logC) + (int64_t)(tid >> lcv) * a.S +
               (int64_t)(tid & ((1u << lcv) - 1u)) * V;
        w.gstep = (int64_t)(kThreads >> lcv) * a.S;
    }
    w.l0 = lds_phys(tid * V, a.pad_shift);
    w.lstep = lds_phys(kThreads * V, a.pad_shift);
    return w;
}

// Scalar tiles as an address walk (NT threads): element
// i = tid + m * NT of tile t lies at global element g0 + m * gstep and at
// LDS element l0 + m * lstep, and a thread's elements are all inside the
// tile's valid columns or all outside (valid).  This holds for contiguous
// tiles, and for row tiles of one hi block (P == 1) whose rows have at most
// NT columns (a thread keeps its column; the planner caps scalar rows at NT
// columns); on the LDS side when every pad period divides NT
// (scalar_walk_ok checks all of it).  The walk replaces a 64-bit row offset
// (with its divisions) per element by one add.
struct ScalarWalk {
    int64_t g0, gstep;
    uint32_t l0, lstep;
    bool valid;
};
template <int NT = kThreads>
__device__ __forceinline__ bool scalar_walk_ok(const PassArgs& a) {
    constexpr int lim = __builtin_ctz(NT);
    for (int k = 0; k < 3; ++k) {
        const int sh = (a.pad_shift >> (8 * k)) & 31;
        if (sh != 31 && sh > lim) return false;
    }
    if (a.mode == kContigScalar) return true;
    return a.mode == kRowScalar && a.P == 1 && a.logC <= lim;
}
template <int NT = kThreads>
__device__ __forceinline__ ScalarWalk scalar_walk(const PassArgs& a, int64_t t, uint32_t tid) {
    ScalarWalk w;
    const uint32_t tileE = ((uint32_t)a.P * (uint32_t)a.G) << a.logC;
    if (a.mode == kContigScalar) {
        w.g0 = t * (int64_t)tileE + tid;
        w.gstep = NT;
        w.valid = true;
    } else {
        // row r = tid >> logC (+ m * NT >> logC), column c = tid & (C - 1)
        const int64_t hb = tile_hb(a, t);
        const int64_t l = t - hb * a.L;
        const uint32_t c = tid & ((1u << a.logC) - 1u);
        w.valid = (int64_t)c < a.S - (l << a.logC);
        w.g0 = hb * ((int64_t)a.G * a.S) + (int64_t)(tid >> a.logC) * a.S + (l << a.logC) + c;
        w.gstep = (int64_t)(NT >> a.logC) * a.S;
    }
    w.l0 = lds_phys(tid, a.pad_shift);
    w.lstep = lds_phys(NT, a.pad_shift);
    return w;
}

// NT: threads of the work-group (every thread takes part); SWALK: scalar
// tiles take their addresses from a ScalarWalk where scalar_walk_ok allows
// it (the walk costs registers beside the general path, so only kernels
// whose tiles are mostly scalar enable it)
template <typename T, typename C, int NT = kThreads, bool SWALK = false>
__device__ __forceinline__ void tile_load(C* lds, const PassArgs& a, const T* __restrict__ in, int64_t t,
                                          uint32_t rows) {
    constexpr int V = Vec16<T>::V;
    const uint32_t tileE = rows << a.logC;
    const bool contig = a.mode == kContigVec || a.mode == kContigScalar;
    const int64_t hb = contig ? 0 : tile_hb(a, t);
    const int64_t l = contig ? 0 : t - hb * a.L;
    if (a.mode == kContigVec || a.mode == kRowVec) {
        const uint32_t nvec = tileE / V;
        for (uint32_t i0 = 0; i0 < nvec; i0 += kLoadBatch * NT) {
            uint4 buf[kLoadBatch];
#pragma unroll
            for (int v = 0; v < kLoadBatch; ++v) {
                const uint32_t i = i0 + threadIdx.x + v * NT;
                if (i < nvec) buf[v] = *reinterpret_cast<const uint4*>(in + vec_offset<T>(a, t, i, hb, l, tileE));
            }
#pragma unroll
            for (int v = 0; v < kLoadBatch; ++v) {
                const uint32_t i = i0 + threadIdx.x + v * NT;
                if (i < nvec) {
                    T vals[V];
                    *reinterpret_cast<uint4*>(vals) = buf[v];
                    const uint32_t ph = lds_phys(i * V, a.pad_shift);
                    if (a.cut >= 0) {  // natural-order mask of the filter
                        const int64_t off = vec_offset<T>(a, t, i, hb, l, tileE);
#pragma unroll
                        for (int e = 0; e < V; ++e) {
                            const bool low = (off + e) % a.N < a.cut;
                            lds[ph + e] = (low != (a.cut_keep_high != 0)) ? to_c(vals[e]) : czero<C>();
                        }
                    } else {
#pragma unroll
                        for (int e = 0; e < V; ++e) lds[ph + e] = to_c(vals[e]);
                    }
                }
            }
        }
    } else if (SWALK && a.cut < 0 && scalar_walk_ok<NT>(a)) {
        const ScalarWalk w = scalar_walk<NT>(a, t, threadIdx.x);
        for (uint32_t i0 = 0, m0 = 0; i0 < tileE; i0 += kLoadBatch * NT, m0 += kLoadBatch) {
            T buf[kLoadBatch];
#pragma unroll
            for (int v = 0; v < kLoadBatch; ++v) {
                const uint32_t i = i0 + threadIdx.x + v * NT;
                if (i < tileE) buf[v] = w.valid ? in[w.g0 + (int64_t)(m0 + v) * w.gstep] : from_c<T>(czero<C>());
            }
#pragma unroll
            for (int v = 0; v < kLoadBatch; ++v) {
                const uint32_t i = i0 + threadIdx.x + v * NT;
                if (i < tileE) lds[w.l0 + (m0 + v) * w.lstep] = to_c(buf[v]);
            }
        }
    } else {
        for (uint32_t i0 = 0; i0 < tileE; i0 += kLoadBatch * NT) {
            T buf[kLoadBatch];
#pragma unroll
            for (int v = 0; v < kLoadBatch; ++v) {
                const uint32_t i = i0 + threadIdx.x + v * NT;
                if (i < tileE) {
                    const int64_t off = elem_offset(a, t, i, hb, l, tileE);
                    if (off >= 0 && (a.cut < 0 || ((off % a.N < a.cut) != (a.cut_keep_high != 0))))
                        buf[v] = in[off];
                    else
                        buf[v] = from_c<T>(czero<C>());
                }
            }
#pragma unroll
            for (int v = 0; v < kLoadBatch; ++v) {
                const uint32_t i = i0 + threadIdx.x + v * NT;
                if (i < tileE) lds[lds_phys(i, a.pad_shift)] = to_c(buf[v]);
            }
        }
    }
}

template <typename T, typename C, bool WALK = false, int NT = kThreads, bool SWALK = false>
__device__ __forceinline__ void tile_store(const C* lds, const PassArgs& a, T* __restrict__ out, int64_t t,
                                           uint32_t rows) {
    constexpr int V = Vec16<T>::V;
    const uint32_t tileE = rows << a.logC;
    const bool contig = a.mode == kContigVec || a.mode == kContigScalar;
    const int64_t hb = contig ? 0 : tile_hb(a, t);
    const int64_t l = contig ? 0 : t - hb * a.L;
    if (a.mode == kContigVec || a.mode == kRowVec) {
        const uint32_t nvec = tileE / V;
        static_assert(!WALK || NT == kThreads, "the address walk assumes kThreads threads");
        if (WALK && vec_walk_ok<T>(a)) {
            const VecWalk w = vec_walk<T>(a, t, threadIdx.x, tileE);
            uint32_t m = 0;
            for (uint32_t i = threadIdx.x; i < nvec; i += kThreads, ++m) {
                T vals[V];
                const uint32_t ph = w.l0 + m * w.lstep;
#pragma unroll
                for (int e = 0; e < V; ++e) vals[e] = from_c<T>(lds[ph + e]);
                gstore16<true>(out + w.g0 + (int64_t)m * w.gstep, *reinterpret_cast<const uint4*>(vals));
            }
            return;
        }
        for (uint32_t i = threadIdx.x; i < nvec; i += NT) {
            T vals[V];
            const uint32_t ph = lds_phys(i * V, a.pad_shift);
#pragma unroll
            for (int e = 0; e < V; ++e) vals[e] = from_c<T>(lds[ph + e]);
            gstore16<true>(out + vec_offset<T>(a, t, i, hb, l, tileE), *reinterpret_cast<const uint4*>(vals));
        }
    } else if (SWALK && scalar_walk_ok<NT>(a)) {
        const ScalarWalk w = scalar_walk<NT>(a, t, threadIdx.x);
        if (w.valid) {
            uint32_t m = 0;
            for (uint32_t i = threadIdx.x; i < tileE; i += NT, ++m)
                out[w.g0 + (int64_t)m * w.gstep] = from_c<T>(lds[w.l0 + m * w.lstep]);
        }
    } else {
        for (uint32_t i = threadIdx.x; i < tileE; i += NT) {
            const int64_t off = elem_offset(a, t, i, hb, l, tileE);
            if (off >= 0) out[off] = from_c<T>(lds[lds_phys(i, a.pad_shift)]);
        }
    }
}

// Kernels with 32-bit compute lanes (float, int32, complex64) whose W fits
// in scalar registers (at most 128 bytes) have the vector registers to spare
// for a prefetch of the next tile; their launches use as many work-groups as
// the device holds at once, each looping over tiles.  (The FP64 kernels
// would spill.)
template <typename C, int B>
constexpr bool pass_prefetches() {
    return B * B * (int)sizeof(C) <= 128 && (sizeof(C) == 4 || std::is_same<C, cf>::value);
}

// The prefetch buffer: 32 dwords per thread, eight 16-byte vectors (vector
// modes) or 32 * 4 / sizeof(T) scalars packed into them (scalar modes, T of
// 4, 8 or 16 bytes).  Item m is always a compile-time index.
constexpr int kPfVec = 8;
template <typename T>
struct PfScalar {
    static constexpr int N = (sizeof(T) == 4 || sizeof(T) == 8 || sizeof(T) == 16) ? 32 * 4 / (int)sizeof(T) : 0;
};
template <typename T, int M>
__device__ __forceinline__ T pf_get(const uint4 (&r)[kPfVec]) {
    constexpr int per = 16 / (int)sizeof(T);
    const uint4 q = r[M / per];
    T out;
    if constexpr (sizeof(T) == 16) {
        out = *reinterpret_cast<const T*>(&q);
    } else if constexpr (sizeof(T) == 8) {
        const uint2 h = (M % 2 == 0) ? make_uint2(q.x, q.y) : make_uint2(q.z, q.w);
        out = *reinterpret_cast<const T*>(&h);
    } else {
        const uint32_t w = (M % 4 == 0) ? q.x : (M % 4 == 1) ? q.y : (M % 4 == 2) ? q.z : q.w;
        out = *reinterpret_cast<const T*>(&w);
    }
    return out;
}
template <typename T, int M>
__device__ __forceinline__ void pf_set(uint4 (&r)[kPfVec], const T& v) {
    constexpr int per = 16 / (int)sizeof(T);
    uint4& q = r[M / per];
    if constexpr (sizeof(T) == 16) {
        q = *reinterpret_cast<const uint4*>(&v);
    } else if constexpr (sizeof(T) == 8) {
        const uint2 h = *reinterpret_cast<const uint2*>(&v);
        if (M % 2 == 0) { q.x = h.x; q.y = h.y; } else { q.z = h.x; q.w = h.y; }
    } else {
        const uint32_t w = *reinterpret_cast<const uint32_t*>(&v);
        if (M % 4 == 0) q.x = w; else if (M % 4 == 1) q.y = w; else if (M % 4 == 2) q.z = w; else q.w = w;
    }
}

template <typename T, typename C, int M = 0>
__device__ __forceinline__ void pf_fetch_scalar(uint4 (&r)[kPfVec], const PassArgs& a, const T* __restrict__ in,
                                                int64_t t, uint32_t tid, int64_t hb, int64_t l, uint32_t tileE) {
    if constexpr (M < PfScalar<T>::N) {
        const uint32_t i = tid + M * kThreads;
        if (i < tileE) {
            const int64_t off = elem_offset(a, t, i, hb, l, tileE);
            pf_set<T, M>(r, off >= 0 ? in[off] : from_c<T>(czero<C>()));
        }
        pf_fetch_scalar<T, C, M + 1>(r, a, in, t, tid, hb, l, tileE);
    }
}
template <typename T, typename C, int M = 0>
__device__ __forceinline__ void pf_fetch_scalar_walk(uint4 (&r)[kPfVec], const T* __restrict__ in, const ScalarWalk& w,
                                                     uint32_t tid, uint32_t tileE) {
    if constexpr (M < PfScalar<T>::N) {
        if (tid + M * kThreads < tileE)
            pf_set<T, M>(r, w.valid ? in[w.g0 + (int64_t)M * w.gstep] : from_c<T>(czero<C>()));
        pf_fetch_scalar_walk<T, C, M + 1>(r, in, w, tid, tileE);
    }
}
template <typename T, typename C, int M = 0>
__device__ __forceinline__ void pf_commit_scalar_walk(C* lds, const uint4 (&r)[kPfVec], uint32_t l0, uint32_t lstep,
                                                      uint32_t tid, uint32_t tileE) {
    if constexpr (M < PfScalar<T>::N) {
        if (tid + M * kThreads < tileE) lds[l0 + M * lstep] = to_c(pf_get<T, M>(r));
        pf_commit_scalar_walk<T, C, M + 1>(lds, r, l0, lstep, tid, tileE);
    }
}
template <typename T, typename C, int M = 0>
__device__ __forceinline__ void pf_commit_scalar(C* lds, const uint4 (&r)[kPfVec], const PassArgs& a, uint32_t tid,
                                                 uint32_t tileE) {
    if constexpr (M < PfScalar<T>::N) {
        const uint32_t i = tid + M * kThreads;
        if (i < tileE) lds[lds_phys(i, a.pad_shift)] = to_c(pf_get<T, M>(r));
        pf_commit_scalar<T, C, M + 1>(lds, r, a, tid, tileE);
    }
}

// Runs stages(lds, rows) on every tile of this work-group (t = blockIdx.x +
// i * gridDim.x), loading and storing through the storage type T (compute
// type C in LDS).  PF: when the work-group has more than one tile, the tile
// fits the prefetch buffer and no filter mask applies, the loads of tile
// t + gridDim.x are in flight into registers while tile t runs its stages
// from LDS, so HBM stays busy through the LDS phases.  WALK: vector tiles
// take their addresses from a VecWalk where vec_walk_ok allows it (costs
// registers in every mode, so only kernels that meet vector tiles enable it).
template <typename T, typename C, bool PF = false, bool WALK = false, bool SWALK = false, typename Stages>
__device__ __forceinline__ void tile_loop(C* lds, const PassArgs& a, Stages&& stages) {
    constexpr int V = Vec16<T>::V;
    const uint32_t rows = (uint32_t)a.P * (uint32_t)a.G;
    const uint32_t tileE = rows << a.logC;
    const T* in = static_cast<const T*>(a.in);
    T* out = static_cast<T*>(a.out);
    const bool vec = a.mode == kContigVec || a.mode == kRowVec;
    const bool contig = a.mode == kContigVec || a.mode == kContigScalar;
    int pf = 0;  // 0: none, 1: vectors, 2: scalars
    if constexpr (PF) {
        if (a.cut < 0 && (int64_t)gridDim.x < a.ntiles) {
            if (vec && tileE / V <= (uint32_t)(kPfVec * kThreads)) pf = 1;
            if (!vec && PfScalar<T>::N > 0 && tileE <= (uint32_t)(PfScalar<T>::N * kThreads)) pf = 2;
        }
    }
    [[maybe_unused]] uint4 r[PF ? kPfVec : 1];
    [[maybe_unused]] const bool walk = WALK && vec && vec_walk_ok<T>(a);
    [[maybe_unused]] const bool swalk = SWALK && !vec && scalar_walk_ok(a);
    // the per-item offsets are recomputed for every tile (an opaque thread
    // index): hoisted out of the tile loop they would hold registers per item
    auto fetch = [&](int64_t t) {
        if constexpr (PF) {
            const int64_t hb = contig ? 0 : tile_hb(a, t);
            const int64_t l = contig ? 0 : t - hb * a.L;
            uint32_t tid = threadIdx.x;
            asm volatile("" : "+v"(tid));
            if (pf == 1 && walk) {
                const VecWalk w = vec_walk<T>(a, t, tid, tileE);
#pragma unroll
                for (int v = 0; v < kPfVec; ++v) {
                    const uint32_t i = tid + v * kThreads;
                    if (i < tileE / V) r[v] = gload16<true>(in + w.g0 + (int64_t)v * w.gstep);
                }
            } else if (pf == 1) {
#pragma unroll
                for (int v = 0; v < kPfVec; ++v) {
                    const uint32_t i = tid + v * kThreads;
                    if (i < tileE / V) r[v] = gload16<true>(in + vec_offset<T>(a, t, i, hb, l, tileE));
                }
            } else if (swalk) {
                pf_fetch_scalar_walk<T, C>(r, in, scalar_walk(a, t, tid), tid, tileE);
            } else {
                pf_fetch_scalar<T, C>(r, a, in, t, tid, hb, l, tileE);
            }
        }
    };
    auto commit = [&]() {
        if constexpr (PF) {
            uint32_t tid = threadIdx.x;
            asm volatile("" : "+v"(tid));
            if (pf == 1) {
                const uint32_t l0 = walk ? lds_phys(tid * V, a.pad_shift) : 0u;
                const uint32_t lstep = lds_phys(kThreads * V, a.pad_shift);
#pragma unroll
                for (int v = 0; v < kPfVec; ++v) {
                    const uint32_t i = tid + v * kThreads;
                    if (i < tileE / V) {
                        T vals[V];
                        *reinterpret_cast<uint4*>(vals) = r[v];
                        const uint32_t ph = walk ? l0 + v * lstep : lds_phys(i * V, a.pad_shift);
#pragma unroll
                        for (int e = 0; e < V; ++e) lds[ph + e] = to_c(vals[e]);
                    }
                }
            } else if (swalk) {
                pf_commit_scalar_walk<T, C>(lds, r, lds_phys(tid, a.pad_shift), lds_phys(kThreads, a.pad_shift), tid,
                                            tileE);
            } else {
                pf_commit_scalar<T, C>(lds, r, a, tid, tileE);
            }
        }
    };
    int64_t t = blockIdx.x;
    if (pf && t < a.ntiles) fetch(t);
    for (; t < a.ntiles; t += gridDim.x) {
        if (pf)
            commit();
        else
            tile_load<T, C, kThreads, SWALK>(lds, a, in, t, rows);
        __syncthreads();
        if (pf && t + gridDim.x < a.ntiles) fetch(t + gridDim.x);
        if (!stages(lds, rows, t)) tile_store<T, C, WALK, kThreads, SWALK>(lds, a, out, t, rows);
        __syncthreads();
    }
}

// W in registers.  Small matrices (<= 64 dwords) are read with uniform
// addresses, which the compiler keeps in SGPRs (a VALU instruction may take one
// SGPR operand).  Larger ones (complex radix 5..8) would spill SGPRs, so they
// are staged through LDS, which places them in VGPRs.
template <typename C, int B>
__device__ __forceinline__ void load_w(C (&w)[B * B], const PassArgs& a) {
    const C* __restrict__ Wg = static_cast<const C*>(a.W);
    if constexpr (B * B * sizeof(C) <= 128) {
#pragma unroll
        for (int r = 0; r < B; ++r)
#pragma unroll
            for (int q = 0; q < B; ++q) w[r * B + q] = a.adjoint ? cconj(Wg[q * B + r]) : Wg[r * B + q];
    } else {
        __shared__ C wl[B * B];
        for (int e = threadIdx.x; e < B * B; e += kThreads) {
            const int r = e / B, q = e % B;
            wl[e] = a.adjoint ? cconj(Wg[q * B + r]) : Wg[e];
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < B * B; ++e) w[e] = wl[e];
    }
}

template <typename T, int B>
__global__ __launch_bounds__(kThreads) void gtt_pass_kernel(PassArgs a) {
    using C = typename Tr<T>::C;
    constexpr int RD = RegDigits<B>::v;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C* lds = reinterpret_cast<C*>(smem_raw);
    C w[B * B];
    load_w<C, B>(w, a);
    // integer radix 2: the Hadamard W runs as butterflies
    bool h2 = false;
    if constexpr (B == 2 && std::is_same<C, uint32_t>::value)
        h2 = w[0] == 1u && w[1] == 1u && w[2] == 1u && w[3] == 0xffffffffu;
    // the address walk and the direct store of the last super-stage only pay
    // where vector tiles occur: power-of-two radices
    constexpr bool kPow2 = (B & (B - 1)) == 0;
    constexpr bool kDirect = kPow2 && std::is_same<T, C>::value;
    [[maybe_unused]] const bool direct =
        kDirect && a.k > 0 &&
        (a.mode == kContigVec ||
         (a.mode == kRowVec && a.P == 1 && (int64_t)a.G * a.S * (int64_t)sizeof(C) < (int64_t(1) << 31))) &&
        (int64_t)a.P * a.G * ((int64_t)sizeof(C) << a.logC) < (int64_t(1) << 31);
    tile_loop<T, C, pass_prefetches<C, B>(), kPow2, !kPow2>(lds, a, [&](C* t, uint32_t rows, int64_t tile) {
        if constexpr (kDirect) {
            if (direct) {
                int64_t gt0 = tile * (int64_t)(rows << a.logC);
                if (a.mode == kRowVec) {
                    const int64_t hb = tile_hb(a, tile);
                    gt0 = hb * ((int64_t)a.G * a.S) + ((tile - hb * a.L) << a.logC);
                }
                run_stages<C, B, RD>(t, a, rows, w, h2, reinterpret_cast<C*>(a.out), gt0);
                return true;
            }
        }
        run_stages<C, B, RD>(t, a, rows, w, h2);
        return false;
    });
}

// ---------------------------------------------------------------------------
// Radix 2, digits 0..k-1 (5 <= k <= 10) of blocks of 2^k contiguous elements
// on wavefronts alone: a wave holds 1024 elements (2^(10-k) blocks), 16 a
// lane; every digit is either a butterfly between two registers of a lane or
// one between two lanes (a cross-lane move).  No LDS, no barriers.
// ---------------------------------------------------------------------------
template <int MASK>
__device__ __forceinline__ uint32_t lane_xor32(uint32_t v) {
    static_assert(MASK == 1 || MASK == 2 || MASK == 4 || MASK == 8, "DPP lane exchange");
    if constexpr (MASK == 1) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);  // quad [1,0,3,2]
    if constexpr (MASK == 2) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);  // quad [2,3,0,1]
    if constexpr (MASK == 4) {  // half-row mirror (lane ^ 7), then quad [3,2,1,0] (lane ^ 3)
        const int t = __builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, false);
        return (uint32_t)__builtin_amdgcn_mov_dpp(t, 0x1B, 0xF, 0xF, false);
    }
    // MASK 8: row mirror (lane ^ 15), then half-row mirror (lane ^ 7)
    const int t = __builtin_amdgcn_mov_dpp((int)v, 0x140, 0xF, 0xF, false);
    return (uint32_t)__builtin_amdgcn_mov_dpp(t, 0x141, 0xF, 0xF, false);
}

// The pair (x_lo, x_hi) of the butterfly across lane bit log2(MASK): the
// values of the lane with that bit clear and of the lane with it set.  Lane
// bits 0-3 move data with DPP (the partner's value, then a select); bits 4
// and 5 with the permlane swaps, which hand every lane both halves at once
// (a swap of a register with a copy of itself leaves the low row or half in
// the first result and the high one in the second).  All VALU: no LDS.
template <int MASK, typename C>
__device__ __forceinline__ void lane_pair(const C& v, bool hi, C& lo_v, C& hi_v) {
    static_assert(sizeof(C) % 4 == 0, "32-bit words");
    constexpr int NW = (int)(sizeof(C) / 4);
    uint32_t w[NW], lo[NW], hw[NW];
    __builtin_memcpy(w, &v, sizeof(C));
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        if constexpr (MASK == 16) {
            const auto r = __builtin_amdgcn_permlane16_swap(w[i], w[i], false, false);
            lo[i] = r[0];
            hw[i] = r[1];
        } else if constexpr (MASK == 32) {
            const auto r = __builtin_amdgcn_permlane32_swap(w[i], w[i], false, false);
            lo[i] = r[0];
            hw[i] = r[1];
        } else {
            const uint32_t p = lane_xor32<MASK>(w[i]);
            lo[i] = hi ? p : w[i];
            hw[i] = hi ? w[i] : p;
        }
    }
    __builtin_memcpy(&lo_v, lo, sizeof(C));
    __builtin_memcpy(&hi_v, hw, sizeof(C));
}

// one digit held across lane bit log2(MASK): the lane with the bit clear keeps
// W[0][0] x_lo + W[0][1] x_hi, the lane with it set W[1][0] x_lo + W[1][1] x_hi
template <int MASK, typename C>
__device__ __forceinline__ void lane_digit(C (&v)[16], const C (&w)[4], uint32_t lane, bool h2) {
    const bool hi = (lane & MASK) != 0;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        C lo_v, hi_v;
        lane_pair<MASK>(v[r], hi, lo_v, hi_v);
        if constexpr (std::is_same<C, uint32_t>::value) {
            if (h2) {  // integer Hadamard: add / subtract
                v[r] = hi ? lo_v - hi_v : lo_v + hi_v;
                continue;
            }
        }
        v[r] = hi ? cmac(cmul(w[2], lo_v), w[3], hi_v) : cmac(cmul(w[0], lo_v), w[1], hi_v);
    }
}

// register digit D of a 16-register block (both the general and the integer
// Hadamard form)
template <typename C, int D>
__device__ __forceinline__ void reg_digit(C (&v)[16], const C (&w)[4], bool h2) {
    if constexpr (std::is_same<C, uint32_t>::value) {
        if (h2) {
            block_digit_h2<C, 4, D>(v);
            return;
        }
    }
    block_digit<C, 2, 4, D>(v, w);
}

// Radix 2 with no LDS and no barrier: one wave holds 1024 elements, 16 per
// lane.  Element i of the wave's block sits in register e + V q of lane l
// where i = e + V (l + 64 q) (V elements per 16-byte vector, e < V): every
// load or store instruction of the wave covers 1 KiB of contiguous memory.
// Digit d of i (the factors act digit by digit, in any order, Eq. (1)) is
// thus register bit d for d < log2 V, lane bit d - log2 V up to log2 V + 5,
// and register bit d - 6 above; the register digits of a k-digit group are
// the low max(log2 V, k - 6) register bits, the lane digits the low
// min(k - log2 V, 6) lane bits.  The grid loops over blocks.
template <typename T>
__global__ __launch_bounds__(kThreads) void gtt_pass_wave2_kernel(PassArgs a) {
    using C = typename Tr<T>::C;
    C w[4];
    load_w<C, 2>(w, a);
    bool h2 = false;
    if constexpr (std::is_same<C, uint32_t>::value)
        h2 = w[0] == 1u && w[1] == 1u && w[2] == 1u && w[3] == 0xffffffffu;
    const int64_t E = a.ntiles * (int64_t)a.P * (int64_t)a.G;
    const T* in = static_cast<const T*>(a.in);
    T* out = static_cast<T*>(a.out);
    const uint32_t lane = threadIdx.x & 63;
    constexpr int V = Vec16<T>::V;  // storage elements per 16-byte vector
    constexpr int LV = V == 1 ? 0 : V == 2 ? 1 : V == 4 ? 2 : 3;
    constexpr int NV = 16 / V;  // vectors per lane
    static_assert((1 << LV) == V && NV * V == 16, "16 elements a lane in whole 16-byte vectors");
    const int rd = a.k - 6 > LV ? a.k - 6 : LV;  // register digits
    const int nl = a.k - LV < 6 ? a.k - LV : 6;  // lane digits
    const int64_t nwaves = (E + 1023) / 1024;
    for (int64_t wv = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6); wv < nwaves;
         wv += (int64_t)gridDim.x * (kThreads / 64)) {
        // E is a multiple of 2^k >= 32 elements: a 16-byte vector is wholly
        // inside or wholly past the end, and a transform vector too (its
        // zero-filled lanes mix only with each other and are not stored)
        const int64_t base = wv * 1024 + (int64_t)lane * V;
        C v[16];
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            const int64_t e0 = base + (int64_t)q * 64 * V;
            if (e0 < E) {
                T vals[V];
                *reinterpret_cast<uint4*>(vals) = gload16<true>(in + e0);
#pragma unroll
                for (int e = 0; e < V; ++e) v[q * V + e] = to_c(vals[e]);
            } else {
#pragma unroll
                for (int e = 0; e < V; ++e) v[q * V + e] = czero<C>();
            }
        }
        // register digits (the same rd and nl in every lane: no divergence)
        if (0 < rd) reg_digit<C, 0>(v, w, h2);
        if (1 < rd) reg_digit<C, 1>(v, w, h2);
        if (2 < rd) reg_digit<C, 2>(v, w, h2);
        if (3 < rd) reg_digit<C, 3>(v, w, h2);
        if (0 < nl) lane_digit<1>(v, w, lane, h2);
        if (1 < nl) lane_digit<2>(v, w, lane, h2);
        if (2 < nl) lane_digit<4>(v, w, lane, h2);
        if (3 < nl) lane_digit<8>(v, w, lane, h2);
        if (4 < nl) lane_digit<16>(v, w, lane, h2);
        if (5 < nl) lane_digit<32>(v, w, lane, h2);
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            const int64_t e0 = base + (int64_t)q * 64 * V;
            if (e0 < E) {
                T vals[V];
#pragma unroll
                for (int e = 0; e < V; ++e) vals[e] = from_c<T>(v[q * V + e]);
                gstore16<true>(out + e0, *reinterpret_cast<const uint4*>(vals));
            }
        }
    }
}

// the wave form applies: radix 2, digits 0..k-1 of contiguous 16-byte-vector
// tiles (groups starting at digit 0), 5 <= k <= 10, no filter mask, 16
// elements a lane in whole 16-byte vectors
template <typename T>
__host__ __device__ inline bool wave2_ok(const PassArgs& a) {
    return a.mode == kContigVec && a.logC == 0 && a.S == 1 && a.k >= 5 && a.k <= 10 && a.cut < 0 &&
           (16 * sizeof(T)) % 16 == 0 && sizeof(T) <= 16;
}

}  // namespace gtt

namespace gtt {

// ---------------------------------------------------------------------------
// Runtime-radix group pass (any radix up to 64, mixed radices allowed): used
// for radices without a specialised kernel and for heterogeneous transforms
// (§2.6, remark on distinct factors).  W matrices are staged in LDS; tiles
// are unpadded (positions linear).  A digit of radix <= 16 runs in place on
// the tile: a thread owns whole fibres, reads the B values of one into
// registers and writes the B results back (code compiled per radix, W read
// from LDS by all lanes at one address).  A larger radix goes out of place,
// element by element, into a second tile buffer that the planner adds.
// ---------------------------------------------------------------------------
template <typename C, int B>
__device__ __forceinline__ void fibre_digit(C* buf, const C* Wj, const PassArgs& a, int j, uint32_t tileE) {
    const uint32_t F = tileE / (uint32_t)B;
    const uint32_t Cm = (1u << a.logC) - 1u;
    const uint32_t pv = (uint32_t)a.bpow[j];
    const uint32_t step = pv << a.logC;
    for (uint32_t f = threadIdx.x; f < F; f += kThreads) {
        const uint32_t c = f & Cm;
        const uint32_t f1 = f >> a.logC;
        const uint32_t Q = fdiv(f1, a.divb[j]);  // f1 / pv
        const uint32_t lo = f1 - Q * pv;
        const uint32_t lam0 = ((Q * pv * (uint32_t)B + lo) << a.logC) | c;
        C* fb = buf + lam0;
        C v[B];
#pragma unroll
        for (int q = 0; q < B; ++q) v[q] = fb[q * step];
#pragma unroll
        for (int r = 0; r < B; ++r) {
            C acc = cmul(Wj[r * B], v[0]);
#pragma unroll
            for (int q = 1; q < B; ++q) acc = cmac(acc, Wj[r * B + q], v[q]);
            fb[r * step] = acc;
        }
    }
}

// the group's digits on a tile in LDS (buf0 holds it on entry); returns the
// buffer holding the result
template <typename C>
__device__ __forceinline__ C* generic_digits(C* buf0, C* buf1, const C* Wl, const PassArgs& a, uint32_t rows) {
    const uint32_t tileE = rows << a.logC;
    const uint32_t Cm = (1u << a.logC) - 1u;
    C* src = buf0;
    C* dst = buf1;
    int woff = 0;
    for (int j = 0; j < a.k; ++j) {
        const int bj = a.rad[j];
        const C* Wj = Wl + woff;
        switch (bj) {
            case 2: fibre_digit<C, 2>(src, Wj, a, j, tileE); break;
            case 3: fibre_digit<C, 3>(src, Wj, a, j, tileE); break;
            case 4: fibre_digit<C, 4>(src, Wj, a, j, tileE); break;
            case 5: fibre_digit<C, 5>(src, Wj, a, j, tileE); break;
            case 6: fibre_digit<C, 6>(src, Wj, a, j, tileE); break;
            case 7: fibre_digit<C, 7>(src, Wj, a, j, tileE); break;
            case 8: fibre_digit<C, 8>(src, Wj, a, j, tileE); break;
            case 9: fibre_digit<C, 9>(src, Wj, a, j, tileE); break;
            case 10: fibre_digit<C, 10>(src, Wj, a, j, tileE); break;
            case 11: fibre_digit<C, 11>(src, Wj, a, j, tileE); break;
            case 12: fibre_digit<C, 12>(src, Wj, a, j, tileE); break;
            case 13: fibre_digit<C, 13>(src, Wj, a, j, tileE); break;
            case 14: fibre_digit<C, 14>(src, Wj, a, j, tileE); break;
            case 15: fibre_digit<C, 15>(src, Wj, a, j, tileE); break;
            case 16: fibre_digit<C, 16>(src, Wj, a, j, tileE); break;
            default: {
                const uint32_t b = (uint32_t)bj;
                const uint32_t pv = (uint32_t)a.bpow[j];
                for (uint32_t i = threadIdx.x; i < tileE; i += kThreads) {
                    const uint32_t c = i & Cm;
                    const uint32_t r = i >> a.logC;
                    const uint32_t hi = fdiv(r, a.divb[j]);              // r / pv
                    const uint32_t d = hi - fdiv(hi, a.divrad[j]) * b;  // digit j of r
                    const uint32_t r0 = r - d * pv;
                    C acc = czero<C>();
                    for (uint32_t q = 0; q < b; ++q)
                        acc = cmac(acc, Wj[d * b + q], src[((r0 + q * pv) << a.logC) | c]);
                    dst[i] = acc;
                }
                C* tmp = src;
                src = dst;
                dst = tmp;
            }
        }
        __syncthreads();
        woff += bj * bj;
    }
    return src;
}

// SW: element-wise tiles take the scalar address walk (costs registers: the
// launch uses this form only for groups whose tiles are element-wise)
template <typename T, bool SW>
__global__ __launch_bounds__(kThreads) void gtt_pass_generic_kernel(PassArgs a) {
    using C = typename Tr<T>::C;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C* Wl = reinterpret_cast<C*>(smem_raw);
    const uint32_t rows = (uint32_t)a.P * (uint32_t)a.G;
    const uint32_t tileE = rows << a.logC;
    const uint32_t wpad = ((uint32_t)a.wtotal + 15u) & ~15u;
    C* buf0 = Wl + wpad;
    C* buf1 = buf0 + lds_tile_elems(tileE, a.pad_shift);  // only for radices above 16
    {
        const C* __restrict__ Wg = static_cast<const C*>(a.W);
        for (int j = 0, done = 0; j < a.k; ++j) {
            // each group digit gets its own copy (offset = running sum)
            const int bj = a.rad[j];
            for (int e = threadIdx.x; e < bj * bj; e += kThreads) {
                const int r = e / bj, q = e - r * bj;
                Wl[done + e] = a.adjoint ? cconj(Wg[a.wofs[j] + q * bj + r]) : Wg[a.wofs[j] + e];
            }
            done += bj * bj;
        }
    }
    for (int64_t t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
        tile_load<T, C, kThreads, SW>(buf0, a, static_cast<const T*>(a.in), t, rows);
        __syncthreads();
        const C* res = generic_digits<C>(buf0, buf1, Wl, a, rows);
        tile_store<T, C, false, kThreads, SW>(res, a, static_cast<T*>(a.out), t, rows);
        __syncthreads();
    }
}

}  // namespace gtt
