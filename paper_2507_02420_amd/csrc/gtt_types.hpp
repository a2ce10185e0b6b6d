// Element types, conversions and multiply-accumulate for the GTT kernels.
//
// Storage types are what lives in HBM; every storage type has a compute type
// (the precision of registers and LDS inside a digit group) and a W type (the
// dtype of the base matrix, equal to the compute type).
//   double -> double          float  -> float
//   cd (complex double)       cf (complex float)
//   bf16 / f16 -> float       int32  -> uint32 (arithmetic mod 2^32)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gtt {

struct alignas(8) cf {  // 8-byte aligned: LDS accesses are single 64-bit operations
    float re, im;
};
struct cd {
    double re, im;
};
struct bf16 {
    uint16_t bits;
};
struct f16 {
    uint16_t bits;
};

template <typename T>
struct Tr;

template <>
struct Tr<float> {
    using C = float;
    static constexpr bool complex = false;
    static constexpr bool integer = false;
};
template <>
struct Tr<double> {
    using C = double;
    static constexpr bool complex = false;
    static constexpr bool integer = false;
};
template <>
struct Tr<cf> {
    using C = cf;
    static constexpr bool complex = true;
    static constexpr bool integer = false;
};
template <>
struct Tr<cd> {
    using C = cd;
    static constexpr bool complex = true;
    static constexpr bool integer = false;
};
template <>
struct Tr<bf16> {
    using C = float;
    static constexpr bool complex = false;
    static constexpr bool integer = false;
};
template <>
struct Tr<f16> {
    using C = float;
    static constexpr bool complex = false;
    static constexpr bool integer = false;
};
template <>
struct Tr<int32_t> {
    using C = uint32_t;
    static constexpr bool complex = false;
    static constexpr bool integer = true;
};

// ---- conversions storage <-> compute ---------------------------------------
__device__ __forceinline__ float to_c(float v) { return v; }
__device__ __forceinline__ double to_c(double v) { return v; }
__device__ __forceinline__ cf to_c(cf v) { return v; }
__device__ __forceinline__ cd to_c(cd v) { return v; }
__device__ __forceinline__ uint32_t to_c(int32_t v) { return (uint32_t)v; }
__device__ __forceinline__ float to_c(bf16 v) { return __uint_as_float(((uint32_t)v.bits) << 16); }
__device__ __forceinline__ float to_c(f16 v) {
    _Float16 h = __builtin_bit_cast(_Float16, v.bits);
    return (float)h;
}

template <typename T>
__device__ __forceinline__ T from_c(typename Tr<T>::C v);
template <>
__device__ __forceinline__ float from_c<float>(float v) { return v; }
template <>
__device__ __forceinline__ double from_c<double>(double v) { return v; }
template <>
__device__ __forceinline__ cf from_c<cf>(cf v) { return v; }
template <>
__device__ __forceinline__ cd from_c<cd>(cd v) { return v; }
template <>
__device__ __forceinline__ int32_t from_c<int32_t>(uint32_t v) { return (int32_t)v; }
template <>
__device__ __forceinline__ bf16 from_c<bf16>(float v) {
    // round to nearest, ties to even (gfx950's v_cvt_pk_bf16_f32); NaN stays
    // a quiet NaN
    bf16 r;
    r.bits = __builtin_bit_cast(uint16_t, (__bf16)v);
    return r;
}
template <>
__device__ __forceinline__ f16 from_c<f16>(float v) {
    _Float16 h = (_Float16)v;  // v_cvt_f16_f32: round to nearest even
    f16 r;
    r.bits = __builtin_bit_cast(uint16_t, h);
    return r;
}

// ---- zero / conj / multiply-accumulate -------------------------------------
template <typename C>
__device__ __forceinline__ C czero();
template <>
__device__ __forceinline__ float czero<float>() { return 0.f; }
template <>
__device__ __forceinline__ double czero<double>() { return 0.0; }
template <>
__device__ __forceinline__ uint32_t czero<uint32_t>() { return 0u; }
template <>
__device__ __forceinline__ cf czero<cf>() { return cf{0.f, 0.f}; }
template <>
__device__ __forceinline__ cd czero<cd>() { return cd{0.0, 0.0}; }

__device__ __forceinline__ float cconj(float v) { return v; }
__device__ __forceinline__ double cconj(double v) { return v; }
__device__ __forceinline__ uint32_t cconj(uint32_t v) { return v; }
__device__ __forceinline__ cf cconj(cf v) { return cf{v.re, -v.im}; }
__device__ __forceinline__ cd cconj(cd v) { return cd{v.re, -v.im}; }

// acc + w * x
__device__ __forceinline__ float cmac(float acc, float w, float x) { return __builtin_fmaf(w, x, acc); }
__device__ __forceinline__ double cmac(double acc, double w, double x) { return __builtin_fma(w, x, acc); }
__device__ __forceinline__ uint32_t cmac(uint32_t acc, uint32_t w, uint32_t x) { return acc + w * x; }
__device__ __forceinline__ cf cmac(cf acc, cf w, cf x) {
    acc.re = __builtin_fmaf(w.re, x.re, acc.re);
    acc.re = __builtin_fmaf(-w.im, x.im, acc.re);
    acc.im = __builtin_fmaf(w.re, x.im, acc.im);
    acc.im = __builtin_fmaf(w.im, x.re, acc.im);
    return acc;
}
__device__ __forceinline__ cd cmac(cd acc, cd w, cd x) {
    acc.re = __builtin_fma(w.re, x.re, acc.re);
    acc.re = __builtin_fma(-w.im, x.im, acc.re);
    acc.im = __builtin_fma(w.re, x.im, acc.im);
    acc.im = __builtin_fma(w.im, x.re, acc.im);
    return acc;
}
// first product (no accumulator): w * x
__device__ __forceinline__ float cmul(float w, float x) { return w * x; }
__device__ __forceinline__ double cmul(double w, double x) { return w * x; }
__device__ __forceinline__ uint32_t cmul(uint32_t w, uint32_t x) { return w * x; }
__device__ __forceinline__ cf cmul(cf w, cf x) {
    cf r;
    r.re = __builtin_fmaf(-w.im, x.im, w.re * x.re);
    r.im = __builtin_fmaf(w.im, x.re, w.re * x.im);
    return r;
}
__device__ __forceinline__ cd cmul(cd w, cd x) {
    cd r;
    r.re = __builtin_fma(-w.im, x.im, w.re * x.re);
    r.im = __builtin_fma(w.im, x.re, w.re * x.im);
    return r;
}

// acc + x * conj(a): the rank-1 update c a^H used by the weight gradient
__device__ __forceinline__ float cmac_conj(float acc, float c, float a) { return __builtin_fmaf(c, a, acc); }
__device__ __forceinline__ double cmac_conj(double acc, double c, double a) { return __builtin_fma(c, a, acc); }
__device__ __forceinline__ cf cmac_conj(cf acc, cf c, cf a) {
    acc.re = __builtin_fmaf(c.re, a.re, acc.re);
    acc.re = __builtin_fmaf(c.im, a.im, acc.re);
    acc.im = __builtin_fmaf(c.im, a.re, acc.im);
    acc.im = __builtin_fmaf(-c.re, a.im, acc.im);
    return acc;
}
__device__ __forceinline__ cd cmac_conj(cd acc, cd c, cd a) {
    acc.re = __builtin_fma(c.re, a.re, acc.re);
    acc.re = __builtin_fma(c.im, a.im, acc.re);
    acc.im = __builtin_fma(c.im, a.re, acc.im);
    acc.im = __builtin_fma(-c.re, a.im, acc.im);
    return acc;
}

__device__ __forceinline__ float cadd(float a, float b) { return a + b; }
__device__ __forceinline__ double cadd(double a, double b) { return a + b; }
__device__ __forceinline__ cf cadd(cf a, cf b) { return cf{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cd cadd(cd a, cd b) { return cd{a.re + b.re, a.im + b.im}; }

// 16-byte global accesses with the non-temporal hint: tile streams that a
// launch reads or writes once
typedef unsigned int ntu32x4 __attribute__((ext_vector_type(4)));
template <bool NT>
__device__ __forceinline__ uint4 gload16(const void* p) {
    if constexpr (NT) {
        const ntu32x4 v = __builtin_nontemporal_load(reinterpret_cast<const ntu32x4*>(p));
        return make_uint4(v[0], v[1], v[2], v[3]);
    } else {
        return *reinterpret_cast<const uint4*>(p);
    }
}
template <bool NT>
__device__ __forceinline__ void gstore16(void* p, uint4 u) {
    if constexpr (NT) {
        ntu32x4 v = {u.x, u.y, u.z, u.w};
        __builtin_nontemporal_store(v, reinterpret_cast<ntu32x4*>(p));
    } else {
        *reinterpret_cast<uint4*>(p) = u;
    }
}

}  // namespace gtt
