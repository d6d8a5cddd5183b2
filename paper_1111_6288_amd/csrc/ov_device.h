// Device-side helpers shared by the libov kernels: complex arithmetic on
// registers, and the three storage formats of spinor and link components.
//
// Internal field layout ("planes"): a spinor field is 12 planes of Vp
// complex numbers, plane k = 3*spin + colour, site index fastest, so that a
// wavefront of 64 consecutive sites reads 64 consecutive complex numbers per
// load.  A batch of fields is a sequence of such fields, `fstride` storage
// elements apart.  Links are 4*9 planes [mu][3*a+b][Vp].  Vp is V rounded up
// to a multiple of 64.  Invariant: the padding sites V..Vp-1 of every field
// hold zeros.  Kernels that reduce or combine whole planes (dots, linear
// combinations, projections) rely on it, so every kernel that writes a field
// writes zeros there (the workspace is reused across precisions and calls).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ov {

template <class R>
struct cx {
    R x, y;
};

template <class R>
__device__ __forceinline__ cx<R> cmk(R a, R b) { return cx<R>{a, b}; }
template <class R>
__device__ __forceinline__ cx<R> cadd(cx<R> a, cx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <class R>
__device__ __forceinline__ cx<R> csub(cx<R> a, cx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <class R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b)
{
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// conj(a) * b
template <class R>
__device__ __forceinline__ cx<R> cmulc(cx<R> a, cx<R> b)
{
    return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
// acc += a * b
template <class R>
__device__ __forceinline__ void cfma(cx<R> &acc, cx<R> a, cx<R> b)
{
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
}
// acc += conj(a) * b
template <class R>
__device__ __forceinline__ void cfmac(cx<R> &acc, cx<R> a, cx<R> b)
{
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(-a.y, b.x, acc.y);
}
template <class R>
__device__ __forceinline__ cx<R> cscale(cx<R> a, R s) { return {a.x * s, a.y * s}; }
// i * a
template <class R>
__device__ __forceinline__ cx<R> cimul(cx<R> a) { return {-a.y, a.x}; }
// -i * a
template <class R>
__device__ __forceinline__ cx<R> cnimul(cx<R> a) { return {a.y, -a.x}; }

// ---------------------------------------------------------------- storage
// double2 (FP64), float2 (FP32) and a packed pair of bfloat16 (re in the low
// half, im in the high half of a 32-bit word).

__device__ __forceinline__ float bf16_lo(uint32_t v) { return __uint_as_float(v << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t v) { return __uint_as_float(v & 0xffff0000u); }

// float -> bfloat16 bits, round to nearest even; NaN stays a quiet NaN.
__device__ __forceinline__ uint32_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0u;
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}

template <class S>
struct StoreT;
template <>
struct StoreT<double2> {
    using real = double;
    static constexpr int bytes = 16;
};
template <>
struct StoreT<float2> {
    using real = float;
    static constexpr int bytes = 8;
};
template <>
struct StoreT<uint32_t> {
    using real = float;
    static constexpr int bytes = 4;
};

template <class R>
__device__ __forceinline__ cx<R> ldc(const double2 *p, long i)
{
    double2 v = p[i];
    return {(R)v.x, (R)v.y};
}
template <class R>
__device__ __forceinline__ cx<R> ldc(const float2 *p, long i)
{
    float2 v = p[i];
    return {(R)v.x, (R)v.y};
}
template <class R>
__device__ __forceinline__ cx<R> ldc(const uint32_t *p, long i)
{
    uint32_t v = p[i];
    return {(R)bf16_lo(v), (R)bf16_hi(v)};
}

template <class R>
__device__ __forceinline__ cx<R> ldc(const double2 *p, unsigned i)
{
    double2 v = p[i];
    return {(R)v.x, (R)v.y};
}
template <class R>
__device__ __forceinline__ cx<R> ldc(const float2 *p, unsigned i)
{
    float2 v = p[i];
    return {(R)v.x, (R)v.y};
}
template <class R>
__device__ __forceinline__ cx<R> ldc(const uint32_t *p, unsigned i)
{
    uint32_t v = p[i];
    return {(R)bf16_lo(v), (R)bf16_hi(v)};
}
template <class R>
__device__ __forceinline__ void stc(double2 *p, unsigned i, cx<R> v)
{
    p[i] = make_double2((double)v.x, (double)v.y);
}
template <class R>
__device__ __forceinline__ void stc(float2 *p, unsigned i, cx<R> v)
{
    p[i] = make_float2((float)v.x, (float)v.y);
}
template <class R>
__device__ __forceinline__ void stc(uint32_t *p, unsigned i, cx<R> v)
{
    p[i] = f2bf((float)v.x) | (f2bf((float)v.y) << 16);
}

template <class R>
__device__ __forceinline__ void stc(double2 *p, long i, cx<R> v)
{
    p[i] = make_double2((double)v.x, (double)v.y);
}
template <class R>
__device__ __forceinline__ void stc(float2 *p, long i, cx<R> v)
{
    p[i] = make_float2((float)v.x, (float)v.y);
}
template <class R>
__device__ __forceinline__ void stc(uint32_t *p, long i, cx<R> v)
{
    p[i] = f2bf((float)v.x) | (f2bf((float)v.y) << 16);
}

// Lattice geometry passed by value to kernels.
struct Geo {
    int Lx, Ly, Lz, Lt;
    int V, Vp;
    int Lxy, Lxyz;
    float bcf[4];   // boundary multiplier on wrapping hops: 1, -1 or 0
};

}  // namespace ov
