// dev.hpp -- device-side building blocks of the staggered operator on gfx950:
// complex and SU(3) arithmetic, the native storage formats of links and
// colour vectors, and the checkerboard geometry with the staggered phases.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lqs {

enum Prec : int { F64 = 0, F32 = 1, F16 = 2 };

typedef _Float16 half_t;

// ---------------------------------------------------------------------------
// complex numbers, colour vectors, SU(3) matrices

template <typename T> struct Cx {
    T re, im;
};

template <typename T> __device__ __forceinline__ Cx<T> cmul(Cx<T> a, Cx<T> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// conj(a) * b
template <typename T> __device__ __forceinline__ Cx<T> cjmul(Cx<T> a, Cx<T> b)
{
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename T> __device__ __forceinline__ Cx<T> cadd(Cx<T> a, Cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> __device__ __forceinline__ Cx<T> csub(Cx<T> a, Cx<T> b) { return {a.re - b.re, a.im - b.im}; }

template <typename T> struct V3 {
    Cx<T> c[3];
};

template <typename T> struct M3 {
    Cx<T> e[3][3];
};

template <typename T> __device__ __forceinline__ M3<T> m3_unit()
{
    M3<T> u;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) u.e[i][j] = {(T)(i == j ? 1 : 0), (T)0};
    return u;
}

template <typename T> __device__ __forceinline__ V3<T> vzero()
{
    V3<T> v;
#pragma unroll
    for (int a = 0; a < 3; ++a) v.c[a] = {T(0), T(0)};
    return v;
}

// The products of the operator are written as explicit fused multiply-adds
// in one fixed order, so that every kernel variant built on them (vectors per
// thread, cached or streaming loads, LDS staging) computes the same bits.
__device__ __forceinline__ float fused(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fused(double a, double b, double c) { return __builtin_fma(a, b, c); }

// U v: each component is sum_b u_ab v_b, accumulated b = 0, 1, 2
template <typename T> __device__ __forceinline__ V3<T> mv(const M3<T> &u, const V3<T> &v)
{
    V3<T> w;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        T re = -(u.e[a][0].im * v.c[0].im), im = u.e[a][0].im * v.c[0].re;
        re = fused(u.e[a][0].re, v.c[0].re, re);
        im = fused(u.e[a][0].re, v.c[0].im, im);
#pragma unroll
        for (int b = 1; b < 3; ++b) {
            re = fused(-u.e[a][b].im, v.c[b].im, fused(u.e[a][b].re, v.c[b].re, re));
            im = fused(u.e[a][b].im, v.c[b].re, fused(u.e[a][b].re, v.c[b].im, im));
        }
        w.c[a] = {re, im};
    }
    return w;
}

// U^dag v: each component is sum_b conj(u_ba) v_b, accumulated b = 0, 1, 2
template <typename T> __device__ __forceinline__ V3<T> mdv(const M3<T> &u, const V3<T> &v)
{
    V3<T> w;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        T re = u.e[0][a].im * v.c[0].im, im = -(u.e[0][a].im * v.c[0].re);
        re = fused(u.e[0][a].re, v.c[0].re, re);
        im = fused(u.e[0][a].re, v.c[0].im, im);
#pragma unroll
        for (int b = 1; b < 3; ++b) {
            re = fused(u.e[b][a].im, v.c[b].im, fused(u.e[b][a].re, v.c[b].re, re));
            im = fused(-u.e[b][a].im, v.c[b].re, fused(u.e[b][a].re, v.c[b].im, im));
        }
        w.c[a] = {re, im};
    }
    return w;
}

// acc += w or acc -= w
template <typename T> __device__ __forceinline__ void accum(V3<T> &acc, const V3<T> &w, bool negate)
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        T re = negate ? -w.c[a].re : w.c[a].re;
        T im = negate ? -w.c[a].im : w.c[a].im;
        acc.c[a].re += re;
        acc.c[a].im += im;
    }
}

// conj(x y - z w), fused in a fixed order like the products above.
template <typename T> __device__ __forceinline__ Cx<T> conj_cross(Cx<T> x, Cx<T> y, Cx<T> z, Cx<T> w)
{
    const T re = fused(x.re, y.re, fused(-x.im, y.im, fused(-z.re, w.re, z.im * w.im)));
    const T im = fused(x.re, y.im, fused(x.im, y.re, fused(-z.re, w.im, -(z.im * w.re))));
    return {re, -im};
}

// Third row of an SU(3) matrix from the first two: row2 = conj(row0 x row1).
template <typename T> __device__ __forceinline__ void rebuild_row2(M3<T> &u)
{
    u.e[2][0] = conj_cross(u.e[0][1], u.e[1][2], u.e[0][2], u.e[1][1]);
    u.e[2][1] = conj_cross(u.e[0][2], u.e[1][0], u.e[0][0], u.e[1][2]);
    u.e[2][2] = conj_cross(u.e[0][0], u.e[1][1], u.e[0][1], u.e[1][0]);
}

// ---------------------------------------------------------------------------
// storage formats
//
// Links of one (direction, parity) block are stored as arrays of Vh words, one
// array after the other ("word-major"), so that a wavefront reading one word
// of consecutive sites touches one contiguous run of memory:
//   F64, 18 reals: 9 x double2 (complex element k = 3*row + col)
//   F64, 12 reals: 6 x double2 (rows 0 and 1)
//   F32, 18 reals: 4 x float4 (elements 0-1, 2-3, 4-5, 6-7) + 1 x float2 (element 8)
//   F32, 12 reals: 3 x float4
//   F16, 18 reals: 2 x 16-byte (elements 0-3, 4-7) + 1 x 4-byte (element 8)
//   F16, 12 reals: 1 x 16-byte (elements 0-3) + 1 x 8-byte (elements 4-5)
// The eight blocks follow each other in the order (mu, parity) = 2*mu + parity.

__host__ __device__ constexpr int link_block_bytes_per_site(int prec, int recon)
{
    return (prec == F64 ? 16 : prec == F32 ? 8 : 4) * (recon == 12 ? 6 : 9);
}

template <int P> struct RealOf { typedef float type; };
template <> struct RealOf<F64> { typedef double type; };

struct alignas(16) W16 { uint32_t w[4]; };
struct alignas(8) W8 { uint32_t w[2]; };

template <typename To, typename From> __device__ __forceinline__ To bitcast(const From &f)
{
    return __builtin_bit_cast(To, f);
}

template <typename T> __device__ __forceinline__ T ldg(const T *p) { return *p; }

// Keeps a load ahead of a branch: its first word becomes an input of an empty
// asm statement, so the load is issued (and waited for) there instead of being
// moved past an early return into the code that uses it.  Loads issued just
// before, such as a gate's state field, then share one memory round trip.
template <typename Raw> __device__ __forceinline__ void issue_here(const Raw &r)
{
    static_assert(sizeof(Raw) >= 4, "a memory word");
    uint32_t w;
    __builtin_memcpy(&w, &r, 4);
    asm volatile("" ::"v"(w));
}

// Streaming loads for the link arrays.  In one operator application every
// link word is used by exactly one thread; when the links are far larger than
// the last-level cache (they are not reused from it across applications
// anyway) they are fetched with the nontemporal hint, so that they do not
// displace the neighbour colour vectors that nearby threads share.
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef float nt_f2 __attribute__((ext_vector_type(2)));
typedef uint32_t nt_u4 __attribute__((ext_vector_type(4)));
typedef uint32_t nt_u2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ld_stream(const double2 *p)
{
    nt_d2 v = __builtin_nontemporal_load((const nt_d2 *)p);
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ float4 ld_stream(const float4 *p)
{
    nt_f4 v = __builtin_nontemporal_load((const nt_f4 *)p);
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ float2 ld_stream(const float2 *p)
{
    nt_f2 v = __builtin_nontemporal_load((const nt_f2 *)p);
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ W16 ld_stream(const W16 *p) { return bitcast<W16>(__builtin_nontemporal_load((const nt_u4 *)p)); }
__device__ __forceinline__ W8 ld_stream(const W8 *p) { return bitcast<W8>(__builtin_nontemporal_load((const nt_u2 *)p)); }
__device__ __forceinline__ uint32_t ld_stream(const uint32_t *p) { return __builtin_nontemporal_load(p); }
template <bool NT, typename T> __device__ __forceinline__ T ld_link(const T *p)
{
    if constexpr (NT) return ld_stream(p);
    else return *p;
}

__device__ __forceinline__ void h8_to_cx(const W16 &w, Cx<float> *out)
{
    struct H8 { half_t h[8]; } h = bitcast<H8>(w);
#pragma unroll
    for (int k = 0; k < 4; ++k) out[k] = {(float)h.h[2 * k], (float)h.h[2 * k + 1]};
}

__device__ __forceinline__ W16 cx_to_h8(const Cx<float> *in)
{
    struct H8 { half_t h[8]; } h;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        h.h[2 * k] = (half_t)in[k].re;
        h.h[2 * k + 1] = (half_t)in[k].im;
    }
    return bitcast<W16>(h);
}

// Load the link of site cb from a (direction, parity) block; the block base
// points at word array 0 and vh is the array length.
template <int P, int R, bool NT = false> struct LinkIO;

// Every format also splits its load into load_raw (the memory words, as
// fetched) and decode (the arithmetic that turns them into the matrix), with
// load = decode(load_raw): a kernel may issue the raw loads of several links
// before decoding any of them and gets the same bits.
template <int R, bool NT> struct LinkIO<F64, R, NT> {
    static constexpr int rows = (R == 12) ? 2 : 3;
    struct Raw { double2 d[3 * rows]; };
    __device__ static __forceinline__ Raw load_raw(const void *base, int64_t vh, int cb)
    {
        const double2 *b = (const double2 *)base;
        Raw r;
#pragma unroll
        for (int k = 0; k < 3 * rows; ++k) r.d[k] = ld_link<NT>(b + k * vh + cb);
        return r;
    }
    __device__ static __forceinline__ M3<double> decode(const Raw &r)
    {
        M3<double> u;
#pragma unroll
        for (int k = 0; k < 3 * rows; ++k) u.e[k / 3][k % 3] = {r.d[k].x, r.d[k].y};
        if (R == 12) rebuild_row2(u);
        return u;
    }
    __device__ static __forceinline__ M3<double> load(const void *base, int64_t vh, int cb)
    {
        return decode(load_raw(base, vh, cb));
    }
    __device__ static __forceinline__ void store(void *base, int64_t vh, int cb, const M3<double> &u)
    {
        double2 *b = (double2 *)base;
        constexpr int rows = (R == 12) ? 2 : 3;
#pragma unroll
        for (int k = 0; k < 3 * rows; ++k) b[k * vh + cb] = make_double2(u.e[k / 3][k % 3].re, u.e[k / 3][k % 3].im);
    }
};

template <int R, bool NT> struct LinkIO<F32, R, NT> {
    static constexpr int n4 = (R == 12) ? 3 : 4;
    struct Raw { float4 d[n4]; float2 t; };
    __device__ static __forceinline__ Raw load_raw(const void *base, int64_t vh, int cb)
    {
        const float4 *b = (const float4 *)base;
        Raw r;
#pragma unroll
        for (int k = 0; k < n4; ++k) r.d[k] = ld_link<NT>(b + k * vh + cb);
        if (R != 12) r.t = ld_link<NT>((const float2 *)(b + 4 * vh) + cb);
        return r;
    }
    __device__ static __forceinline__ M3<float> decode(const Raw &r)
    {
        M3<float> u;
#pragma unroll
        for (int k = 0; k < n4; ++k) {
            u.e[(2 * k) / 3][(2 * k) % 3] = {r.d[k].x, r.d[k].y};
            u.e[(2 * k + 1) / 3][(2 * k + 1) % 3] = {r.d[k].z, r.d[k].w};
        }
        if (R == 12) rebuild_row2(u);
        else u.e[2][2] = {r.t.x, r.t.y};
        return u;
    }
    __device__ static __forceinline__ M3<float> load(const void *base, int64_t vh, int cb)
    {
        return decode(load_raw(base, vh, cb));
    }
    __device__ static __forceinline__ void store(void *base, int64_t vh, int cb, const M3<float> &u)
    {
        float4 *b = (float4 *)base;
        constexpr int n4 = (R == 12) ? 3 : 4;
#pragma unroll
        for (int k = 0; k < n4; ++k) {
            Cx<float> a = u.e[(2 * k) / 3][(2 * k) % 3], c = u.e[(2 * k + 1) / 3][(2 * k + 1) % 3];
            b[k * vh + cb] = make_float4(a.re, a.im, c.re, c.im);
        }
        if (R != 12) {
            float2 *t = (float2 *)(b + 4 * vh);
            t[cb] = make_float2(u.e[2][2].re, u.e[2][2].im);
        }
    }
};

template <int R, bool NT> struct LinkIO<F16, R, NT> {
    // 12 reals: one 16-byte and one 8-byte word; 18: two 16-byte words and 4 bytes
    struct Raw { W16 a; W16 b; W8 c; uint32_t t; };
    __device__ static __forceinline__ Raw load_raw(const void *base, int64_t vh, int cb)
    {
        const W16 *b = (const W16 *)base;
        Raw r;
        r.a = ld_link<NT>(b + cb);
        if (R == 12) {
            r.c = ld_link<NT>((const W8 *)(b + vh) + cb);
        } else {
            r.b = ld_link<NT>(b + vh + cb);
            r.t = ld_link<NT>((const uint32_t *)(b + 2 * vh) + cb);
        }
        return r;
    }
    __device__ static __forceinline__ M3<float> decode(const Raw &r)
    {
        M3<float> u;
        Cx<float> e[9];
        h8_to_cx(r.a, e);
        if (R == 12) {
            struct H4 { half_t h[4]; } h = bitcast<H4>(r.c);
            e[4] = {(float)h.h[0], (float)h.h[1]};
            e[5] = {(float)h.h[2], (float)h.h[3]};
        } else {
            h8_to_cx(r.b, e + 4);
            struct H2 { half_t h[2]; } h = bitcast<H2>(r.t);
            e[8] = {(float)h.h[0], (float)h.h[1]};
        }
        constexpr int n = (R == 12) ? 6 : 9;
#pragma unroll
        for (int k = 0; k < n; ++k) u.e[k / 3][k % 3] = e[k];
        if (R == 12) rebuild_row2(u);
        return u;
    }
    __device__ static __forceinline__ M3<float> load(const void *base, int64_t vh, int cb)
    {
        return decode(load_raw(base, vh, cb));
    }
    __device__ static __forceinline__ void store(void *base, int64_t vh, int cb, const M3<float> &u)
    {
        W16 *b = (W16 *)base;
        Cx<float> e[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) e[k] = u.e[k / 3][k % 3];
        b[cb] = cx_to_h8(e);
        if (R == 12) {
            struct H4 { half_t h[4]; } h;
            h.h[0] = (half_t)e[4].re;
            h.h[1] = (half_t)e[4].im;
            h.h[2] = (half_t)e[5].re;
            h.h[3] = (half_t)e[5].im;
            ((W8 *)(b + vh))[cb] = bitcast<W8>(h);
        } else {
            b[vh + cb] = cx_to_h8(e + 4);
            struct H2 { half_t h[2]; } h;
            h.h[0] = (half_t)e[8].re;
            h.h[1] = (half_t)e[8].im;
            ((uint32_t *)(b + 2 * vh))[cb] = bitcast<uint32_t>(h);
        }
    }
};

// Colour vectors of one parity and one right-hand side (see lqs.h):
//   F64: double2 [3][Vh]; F32: float4 [Vh] + float2 [Vh]; F16: 16-byte [Vh]
//   (six binary16 scaled by a float per site).
__host__ __device__ constexpr int64_t spinor_bytes_per_site(int prec)
{
    return prec == F64 ? 48 : prec == F32 ? 24 : 16;
}

template <int P> struct SpinorIO;

template <> struct SpinorIO<F64> {
    struct Raw { double2 d[3]; };
    __device__ static __forceinline__ Raw load_raw(const void *base, int64_t vh, int cb)
    {
        const double2 *b = (const double2 *)base;
        Raw r;
#pragma unroll
        for (int a = 0; a < 3; ++a) r.d[a] = ldg(b + a * vh + cb);
        return r;
    }
    __device__ static __forceinline__ V3<double> decode(const Raw &r)
    {
        V3<double> v;
#pragma unroll
        for (int a = 0; a < 3; ++a) v.c[a] = {r.d[a].x, r.d[a].y};
        return v;
    }
    __device__ static __forceinline__ V3<double> load(const void *base, int64_t vh, int cb)
    {
        return decode(load_raw(base, vh, cb));
    }
    __device__ static __forceinline__ void store(void *base, int64_t vh, int cb, const V3<double> &v)
    {
        double2 *b = (double2 *)base;
#pragma unroll
        for (int a = 0; a < 3; ++a) b[a * vh + cb] = make_double2(v.c[a].re, v.c[a].im);
    }
};

template <> struct SpinorIO<F32> {
    struct Raw { float4 d; float2 e; };
    __device__ static __forceinline__ Raw load_raw(const void *base, int64_t vh, int cb)
    {
        const float4 *b = (const float4 *)base;
        return {ldg(b + cb), ldg((const float2 *)(b + vh) + cb)};
    }
    __device__ static __forceinline__ V3<float> decode(const Raw &r)
    {
        V3<float> v;
        v.c[0] = {r.d.x, r.d.y};
        v.c[1] = {r.d.z, r.d.w};
        v.c[2] = {r.e.x, r.e.y};
        return v;
    }
    __device__ static __forceinline__ V3<float> load(const void *base, int64_t vh, int cb)
    {
        return decode(load_raw(base, vh, cb));
    }
    __device__ static __forceinline__ void store(void *base, int64_t vh, int cb, const V3<float> &v)
    {
        float4 *b = (float4 *)base;
        b[cb] = make_float4(v.c[0].re, v.c[0].im, v.c[1].re, v.c[1].im);
        ((float2 *)(b + vh))[cb] = make_float2(v.c[2].re, v.c[2].im);
    }
};

// binary16 of a binary32 value held in a register.  The empty asm keeps the
// compiler from folding the multiply that produced x and this conversion into
// one mixed-precision instruction that rounds once: it does so in some kernels
// and not in others, and the colour-vector store and the in-register round trip
// below must round identically (binary32, then binary16) everywhere.
__device__ __forceinline__ half_t to_half(float x)
{
    asm volatile("" : "+v"(x));
    return (half_t)x;
}

struct alignas(16) SpH {
    half_t h[6];
    float s;
};

template <> struct SpinorIO<F16> {
    typedef W16 Raw;
    __device__ static __forceinline__ Raw load_raw(const void *base, int64_t vh, int cb)
    {
        (void)vh;
        return ldg((const W16 *)base + cb);
    }
    __device__ static __forceinline__ V3<float> decode(const Raw &w)
    {
        SpH q = bitcast<SpH>(w);
        V3<float> v;
#pragma unroll
        for (int a = 0; a < 3; ++a) v.c[a] = {(float)q.h[2 * a] * q.s, (float)q.h[2 * a + 1] * q.s};
        return v;
    }
    __device__ static __forceinline__ V3<float> load(const void *base, int64_t vh, int cb)
    {
        return decode(load_raw(base, vh, cb));
    }
    // Scale = max |component| of the site; components stored as binary16 of
    // value / scale (round to nearest even); an all-zero site stores scale 0.
    // value * (1 / scale) is rounded to binary32 and then to binary16 (to_half).
    __device__ static __forceinline__ void store(void *base, int64_t vh, int cb, const V3<float> &v)
    {
        (void)vh;
        float m = 0.f;
#pragma unroll
        for (int a = 0; a < 3; ++a) m = fmaxf(m, fmaxf(fabsf(v.c[a].re), fabsf(v.c[a].im)));
        float inv = m > 0.f ? 1.0f / m : 0.f;
        SpH q;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            q.h[2 * a] = to_half(v.c[a].re * inv);
            q.h[2 * a + 1] = to_half(v.c[a].im * inv);
        }
        q.s = m;
        ((W16 *)base)[cb] = bitcast<W16>(q);
    }
};

// The value a store followed by a load of the given format returns, computed
// in registers with the same operations (so an operand formed on the fly
// equals the stored one bit for bit).
template <int P> struct Roundtrip {
    template <typename T> __device__ static __forceinline__ V3<T> apply(const V3<T> &v) { return v; }
};
template <> struct Roundtrip<F16> {
    __device__ static __forceinline__ V3<float> apply(const V3<float> &v)
    {
        float m = 0.f;
#pragma unroll
        for (int a = 0; a < 3; ++a) m = fmaxf(m, fmaxf(fabsf(v.c[a].re), fabsf(v.c[a].im)));
        const float inv = m > 0.f ? 1.0f / m : 0.f;
        V3<float> w;
#pragma unroll
        for (int a = 0; a < 3; ++a)
            w.c[a] = {(float)to_half(v.c[a].re * inv) * m, (float)to_half(v.c[a].im * inv) * m};
        return w;
    }
};

// ---------------------------------------------------------------------------
// FP16 storage: products on the stored binary16 pairs
//
// A stored complex binary16 number is one 32-bit word, real part in the low
// half.  v_dot2_f32_f16 forms lo*lo + hi*hi + c; binary16 products are exact
// in binary32, so the arithmetic is binary32 as in the decoded form, without
// converting the operands first.  A complex product takes two dot2, the signs
// and the order of the halves set by one bit operation on the vector word.
typedef _Float16 hpair __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float dot2(uint32_t a, uint32_t b, float c)
{
    return __builtin_amdgcn_fdot2(bitcast<hpair>(a), bitcast<hpair>(b), c, false);
}
// dot2(a, b, 0): the three-operand encoding with the constant 0, where the
// compiler would pick the accumulating two-operand form and first move a
// zero into the destination (one extra instruction per chain).
__device__ __forceinline__ float dot2z(uint32_t a, uint32_t b)
{
    float r;
    asm("v_dot2_f32_f16 %0, %1, %2, 0" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ uint32_t swap_h(uint32_t w) { return __builtin_amdgcn_alignbit(w, w, 16); }
constexpr uint32_t NEG_HI = 0x80000000u, NEG_LO = 0x00008000u, NEG_BOTH = 0x80008000u;
__device__ __forceinline__ uint32_t pack_h(float re, float im)
{
    struct P { half_t lo, hi; } p = {to_half(re), to_half(im)};
    return bitcast<uint32_t>(p);
}

// An SU(3) matrix as binary16 pair words e[row][col].  With 12 stored reals
// the rebuilt third row is e[2][b] + lo[b]: its binary32 value rounded to
// binary16 and the rounding remainder, again in binary16 (about 22 bits
// together, where the third row alone in binary16 made some mixed solves
// take 3-6 % more iterations).
struct M3H {
    uint32_t e[3][3];
    uint32_t lo[3];
};

// conj(x y - z w) from pair words: binary32 sums of the exact products, in a
// fixed order, as binary16 pair words hi + lo.
__device__ __forceinline__ void conj_cross_h(uint32_t x, uint32_t y, uint32_t z, uint32_t w, uint32_t &hi, uint32_t &lo)
{
    const float re = dot2(z, w ^ NEG_LO, dot2z(x, y ^ NEG_HI));              // xr yr - xi yi - zr wr + zi wi
    const float nim = dot2(z, swap_h(w), dot2z(x ^ NEG_BOTH, swap_h(y)));  // -(xr yi + xi yr) + zr wi + zi wr
    const hpair h = {(half_t)re, (half_t)nim};
    const hpair l = {(half_t)(re - (float)h.x), (half_t)(nim - (float)h.y)};
    hi = bitcast<uint32_t>(h);
    lo = bitcast<uint32_t>(l);
}

// The link words of LinkIO<F16, R>::Raw as a matrix; with 12 reals the third
// row is rebuilt as conj(row0 x row1).
template <int R, typename Raw> __device__ __forceinline__ M3H link_words(const Raw &r)
{
    M3H u;
    u.e[0][0] = r.a.w[0];
    u.e[0][1] = r.a.w[1];
    u.e[0][2] = r.a.w[2];
    u.e[1][0] = r.a.w[3];
    if constexpr (R == 12) {
        u.e[1][1] = r.c.w[0];
        u.e[1][2] = r.c.w[1];
        conj_cross_h(u.e[0][1], u.e[1][2], u.e[0][2], u.e[1][1], u.e[2][0], u.lo[0]);
        conj_cross_h(u.e[0][2], u.e[1][0], u.e[0][0], u.e[1][2], u.e[2][1], u.lo[1]);
        conj_cross_h(u.e[0][0], u.e[1][1], u.e[0][1], u.e[1][0], u.e[2][2], u.lo[2]);
    } else {
        u.e[1][1] = r.b.w[0];
        u.e[1][2] = r.b.w[1];
        u.e[2][0] = r.b.w[2];
        u.e[2][1] = r.b.w[3];
        u.e[2][2] = r.t;
    }
    return u;
}

// acc += f U v (FWD) or acc += f U^dag v, for the stored FP16 colour vector w
// (three pair words and the site scale) and f = +-scale.  Component a sums its
// three terms b = 0, 1, 2 in dot2 order (a third-row element of a 12-real
// link as its hi part, then its lo part), then one fused multiply-add by f.
//   U v:      re = dot2(u_ab, (vr, -vi)),  im = dot2(u_ab, (vi, vr))
//   U^dag v:  re = dot2(u_ba, (vr, vi)),   im = dot2(u_ba, (vi, -vr))
template <bool FWD, int R>
__device__ __forceinline__ void accum_h(V3<float> &acc, const M3H &u, const W16 &w, bool negate)
{
    uint32_t x[3], y[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        x[b] = FWD ? (w.w[b] ^ NEG_HI) : w.w[b];
        y[b] = FWD ? swap_h(w.w[b]) : (swap_h(w.w[b]) ^ NEG_HI);
    }
    const float sc = bitcast<float>(w.w[3]);
    const float f = negate ? -sc : sc;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const uint32_t m0 = FWD ? u.e[a][0] : u.e[0][a];
        float re = dot2z(m0, x[0]), im = dot2z(m0, y[0]);
        if (R == 12 && FWD && a == 2) {
            re = dot2(u.lo[0], x[0], re);
            im = dot2(u.lo[0], y[0], im);
        }
#pragma unroll
        for (int b = 1; b < 3; ++b) {
            const uint32_t m = FWD ? u.e[a][b] : u.e[b][a];
            re = dot2(m, x[b], re);
            im = dot2(m, y[b], im);
            if (R == 12 && (FWD ? a == 2 : b == 2)) {
                const uint32_t l = u.lo[FWD ? b : a];
                re = dot2(l, x[b], re);
                im = dot2(l, y[b], im);
            }
        }
        acc.c[a].re = fused(f, re, acc.c[a].re);
        acc.c[a].im = fused(f, im, acc.c[a].im);
    }
}

// Convert a vector between real types.
template <typename To, typename From> __device__ __forceinline__ V3<To> vcast(const V3<From> &v)
{
    V3<To> w;
#pragma unroll
    for (int a = 0; a < 3; ++a) w.c[a] = {(To)v.c[a].re, (To)v.c[a].im};
    return w;
}

// ---------------------------------------------------------------------------
// geometry: checkerboard index <-> coordinates, neighbours, staggered phases

struct Geom {
    int32_t n[4];   // Nx, Ny, Nz, Nt
    int32_t vh;     // sites per parity
};

struct Site {
    int32_t lex;        // lexicographic index
    int32_t fwd[4];     // checkerboard index of x + mu
    int32_t bwd[4];     // checkerboard index of x - mu
    uint32_t negf;      // bit mu: phase of link (x, mu) is -1
    uint32_t negb;      // bit mu: phase of link (x - mu, mu) is -1
    uint32_t tunit;     // temporal gauge: bit 0 link (x, t) = 1, bit 1 link (x - t, t) = 1
};

// Lexicographic index of the site with checkerboard index cb and the given parity.
__device__ __forceinline__ int lex_of(const Geom &g, int cb, int parity)
{
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    int lex0 = 2 * cb;
    int q = lex0 / nx;
    int y = q % ny;
    q /= ny;
    int z = q % nz;
    int t = q / nz;
    return lex0 + ((y + z + t + parity) & 1);
}

// Coordinates of the site with checkerboard index cb and the given parity,
// its eight neighbours and the signs of the eight links that touch it.
__device__ __forceinline__ Site decode(const Geom &g, int cb, int parity)
{
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2], nt = g.n[3];
    int lex0 = 2 * cb;
    int q = lex0 / nx;
    int x0 = lex0 - q * nx;
    int y = q % ny;
    q /= ny;
    int z = q % nz;
    int t = q / nz;
    int x = x0 + ((y + z + t + parity) & 1);
    int lex = lex0 + (x - x0);
    const int sy = nx, sz = nx * ny, st = nx * ny * nz;
    Site s;
    s.lex = lex;
    s.fwd[0] = (x == nx - 1 ? lex - (nx - 1) : lex + 1) >> 1;
    s.bwd[0] = (x == 0 ? lex + (nx - 1) : lex - 1) >> 1;
    s.fwd[1] = (y == ny - 1 ? lex - (ny - 1) * sy : lex + sy) >> 1;
    s.bwd[1] = (y == 0 ? lex + (ny - 1) * sy : lex - sy) >> 1;
    s.fwd[2] = (z == nz - 1 ? lex - (nz - 1) * sz : lex + sz) >> 1;
    s.bwd[2] = (z == 0 ? lex + (nz - 1) * sz : lex - sz) >> 1;
    s.fwd[3] = (t == nt - 1 ? lex - (nt - 1) * st : lex + st) >> 1;
    s.bwd[3] = (t == 0 ? lex + (nt - 1) * st : lex - st) >> 1;
    // eta_0 = 1, eta_1 = (-1)^x, eta_2 = (-1)^(x+y), eta_3 = (-1)^(x+y+z);
    // eta_mu does not depend on x_mu, so the backward link shares it, and the
    // antiperiodic sign sits on t-links leaving t = Nt - 1.
    uint32_t e1 = x & 1, e2 = (x + y) & 1, e3 = (x + y + z) & 1;
    uint32_t eta = (e1 << 1) | (e2 << 2) | (e3 << 3);
    s.negf = eta ^ ((t == nt - 1) ? 8u : 0u);
    s.negb = eta ^ ((t == 0) ? 8u : 0u);
    // in temporal gauge every t-link is the unit matrix except those leaving t = Nt - 1
    s.tunit = (t < nt - 1 ? 1u : 0u) | (t > 0 ? 2u : 0u);
    return s;
}

// ---------------------------------------------------------------------------
// reductions (wave64 shuffles, then LDS across the waves of a block)

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over the block; the result is valid in every thread.  blockDim.x must
// be a multiple of 64 and at most 1024.  Fixed order, hence deterministic.
__device__ __forceinline__ double block_sum(double v)
{
    __shared__ double red[16];
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[w];
    return s;
}

// Fixed-order sum of n partials by one block (valid in every thread); the
// loads are device-coherent, for partials written by other blocks of the
// same kernel behind a grid barrier.
__device__ __forceinline__ double sum_partials(const double *p, int n)
{
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += __hip_atomic_load(p + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return block_sum(s);
}

}  // namespace lqs
