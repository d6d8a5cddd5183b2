// Device-side helpers shared by the libov kernels: complex arithmetic on
// registers, and the three storage formats of spinor and link components.
//
// Internal field layout ("planes"): a spinor field is 12 planes of Vp
// complex numbers, plane k = 3*spin + colour, site index fastest, so that a
// wavefront of 64 consecutive sites reads 64 consecutive elements per load
// (FP32 fields pair planes 2p and 2p+1 into 16-byte elements; cpos below).  A batch of fields is a sequence of such fields, `fstride` storage
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

// ---------------------------------------------------------------- layouts
// Position of complex component k (0..11) of site `site` inside a field, in
// units of one stored complex number.  FP64 and BF16 fields are 12 planes of
// one complex per site (16-byte and 4-byte lanes).  FP32 fields pair the
// components: pair-plane p holds (k = 2p, 2p+1) of a site in one 16-byte
// element, because on gfx950 a load of 8 bytes per lane costs as many
// address cycles as one of 16 bytes.  Both layouts keep spins 0,1 (k < 6) in
// the first half of the field, so flat elementwise kernels and gamma5 (negate
// the second half) work on either.
//
// Links: FP64 and BF16 use 36 planes [mu][3a+b][Vp]; FP32 stores, per mu,
// the pairs (0,1) (2,3) (4,5) (6,7) as four pair-planes followed by a plain
// plane for component 8, in the same 9 Vp complex numbers per mu.
template <class S>
struct Pair {
    static constexpr int E = 1;
};
template <>
struct Pair<float2> {
    static constexpr int E = 2;
};

template <class S>
__host__ __device__ __forceinline__ long cpos(int k, long site, long Vp)
{
    if (Pair<S>::E == 2) return 2 * ((k >> 1) * Vp + site) + (k & 1);
    return k * Vp + site;
}

template <class S>
__host__ __device__ __forceinline__ long lpos(int mu, int k, long site, long Vp)
{
    if (Pair<S>::E == 2 && k < 8) return mu * 9 * Vp + 2 * ((k >> 1) * Vp + site) + (k & 1);
    return (mu * 9 + k) * Vp + site;
}

// Mixed-layout traversal: pair-plane p (0..5) and offset r (0..2Vp-1) name
// the same complex number in both layouts; these give its position.
template <class S>
__device__ __forceinline__ long ppos(int p, long r, long Vp)
{
    if (Pair<S>::E == 2) return 2 * p * Vp + r;
    return (2 * p + (r & 1)) * Vp + (r >> 1);
}

// Lattice geometry passed by value to kernels.
struct Geo {
    int Lx, Ly, Lz, Lt;
    int V, Vp;
    int Lxy, Lxyz;
    float bcf[4];   // boundary multiplier on wrapping hops: 1, -1 or 0
};

}  // namespace ov
