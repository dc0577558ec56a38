// pack.hip -- layout conversions: canonical complex128 links into the native
// word-major formats (FP64/FP32/FP16, 18 or 12 reals; the 12-real form keeps
// rows 0 and 1 and the kernels rebuild row 2, Sec. 4.3), canonical colour
// vectors into native single-parity fields and back, and precision changes
// between native fields.  All are one thread per site, once per call.
#include "lqs_impl.hpp"

namespace lqs {

// ---------------------------------------------------------------------------
// the unit link stored at index vh (a padding site) of the two t-link blocks
// of a temporal-gauge format: the hop reads it in place of a unit t-link by
// changing only the site index, so skipping those links needs no branch
// around the product and no second base address

template <int P, int R> __global__ void unit_link_kernel(char *links, int64_t block_bytes, int64_t pitch, int vh)
{
    const M3<typename RealOf<P>::type> u = m3_unit<typename RealOf<P>::type>();
    LinkIO<P, R>::store(links + (6 + threadIdx.x) * block_bytes, pitch, vh, u);
}

void launch_unit_link(const Geom &g, int prec, int recon, int64_t pitch, void *links, hipStream_t s)
{
    LQS_REQUIRE(pitch > g.vh, LQS_EINVAL, "temporal-gauge link planes need a padding site");
    const int64_t bb = (int64_t)link_block_bytes_per_site(prec, recon) * pitch;
    char *l = (char *)links;
#define LQS_UNIT(P, R) hipLaunchKernelGGL((unit_link_kernel<P, R>), dim3(1), dim3(2), 0, s, l, bb, pitch, (int)g.vh)
    if (prec == F64 && recon == 18) LQS_UNIT(F64, 18);
    else if (prec == F64) LQS_UNIT(F64, 12);
    else if (prec == F32 && recon == 18) LQS_UNIT(F32, 18);
    else if (prec == F32) LQS_UNIT(F32, 12);
    else if (recon == 18) LQS_UNIT(F16, 18);
    else LQS_UNIT(F16, 12);
#undef LQS_UNIT
    LQS_HIP(hipGetLastError());
}


template <int P, int R>
__global__ void pack_links_kernel(Geom g, const double2 *canon, char *out, int64_t block_bytes, int64_t pitch)
{
    typedef typename RealOf<P>::type T;
    const int64_t V = 2 * (int64_t)g.vh;
    const int cb = blockIdx.x * blockDim.x + threadIdx.x;
    const int mu = blockIdx.y >> 1, parity = blockIdx.y & 1;
    if (cb >= g.vh) return;
    const int lex = lex_of(g, cb, parity);
    const double2 *src = canon + 9 * ((int64_t)mu * V + lex);
    M3<T> u;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        double2 d = src[k];
        u.e[k / 3][k % 3] = {(T)d.x, (T)d.y};
    }
    LinkIO<P, R>::store(out + (2 * mu + parity) * block_bytes, pitch, cb, u);
}

template <int P, int R>
static void pack_links_t(const Geom &g, const double *canon, int64_t pitch, void *out, hipStream_t s)
{
    const int64_t block_bytes = (int64_t)link_block_bytes_per_site(P, R) * pitch;
    dim3 grid((g.vh + 255) / 256, 8);
    hipLaunchKernelGGL((pack_links_kernel<P, R>), grid, dim3(256), 0, s, g, (const double2 *)canon, (char *)out,
                       block_bytes, pitch);
    LQS_HIP(hipGetLastError());
}

void launch_pack_links(const Geom &g, const double *canon, int prec, int recon, int64_t pitch, void *out,
                       hipStream_t s)
{
    LQS_REQUIRE(pitch >= g.vh, LQS_EINVAL, "link plane pitch below the site count");
    if (prec == F64 && recon == 18) pack_links_t<F64, 18>(g, canon, pitch, out, s);
    else if (prec == F64) pack_links_t<F64, 12>(g, canon, pitch, out, s);
    else if (prec == F32 && recon == 18) pack_links_t<F32, 18>(g, canon, pitch, out, s);
    else if (prec == F32) pack_links_t<F32, 12>(g, canon, pitch, out, s);
    else if (recon == 18) pack_links_t<F16, 18>(g, canon, pitch, out, s);
    else pack_links_t<F16, 12>(g, canon, pitch, out, s);
}

// ---------------------------------------------------------------------------

template <int P>
__global__ void field_pack_kernel(Geom g, const double2 *lex, int parity, char *out, int64_t rhs_stride)
{
    typedef typename RealOf<P>::type T;
    const int64_t V = 2 * (int64_t)g.vh;
    const int cb = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (cb >= g.vh) return;
    const int l = lex_of(g, cb, parity);
    const double2 *src = lex + 3 * (r * V + l);
    V3<T> v;
#pragma unroll
    for (int a = 0; a < 3; ++a) v.c[a] = {(T)src[a].x, (T)src[a].y};
    SpinorIO<P>::store(out + r * rhs_stride, g.vh, cb, v);
}

template <int P>
__global__ void field_unpack_kernel(Geom g, const char *in, int64_t rhs_stride, int parity, double scale,
                                    double2 *lex)
{
    const int64_t V = 2 * (int64_t)g.vh;
    const int cb = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (cb >= g.vh) return;
    const int l = lex_of(g, cb, parity);
    const auto v = SpinorIO<P>::load(in + r * rhs_stride, g.vh, cb);
    double2 *dst = lex + 3 * (r * V + l);
#pragma unroll
    for (int a = 0; a < 3; ++a) dst[a] = make_double2(scale * (double)v.c[a].re, scale * (double)v.c[a].im);
}

void launch_field_pack(const Geom &g, const double *lex, const lqs_field &out, hipStream_t s)
{
    dim3 grid((g.vh + 255) / 256, out.nrhs);
    const int64_t stride = field_bytes(g, out.prec, 1);
    if (out.prec == F64)
        hipLaunchKernelGGL(field_pack_kernel<F64>, grid, dim3(256), 0, s, g, (const double2 *)lex, out.parity,
                           (char *)out.data, stride);
    else if (out.prec == F32)
        hipLaunchKernelGGL(field_pack_kernel<F32>, grid, dim3(256), 0, s, g, (const double2 *)lex, out.parity,
                           (char *)out.data, stride);
    else
        hipLaunchKernelGGL(field_pack_kernel<F16>, grid, dim3(256), 0, s, g, (const double2 *)lex, out.parity,
                           (char *)out.data, stride);
    LQS_HIP(hipGetLastError());
}

// scale 1 leaves every value unchanged (an exact product)
void launch_field_unpack(const Geom &g, const lqs_field &in, double scale, double *lex, hipStream_t s)
{
    dim3 grid((g.vh + 255) / 256, in.nrhs);
    const int64_t stride = field_bytes(g, in.prec, 1);
    if (in.prec == F64)
        hipLaunchKernelGGL(field_unpack_kernel<F64>, grid, dim3(256), 0, s, g, (const char *)in.data, stride,
                           in.parity, scale, (double2 *)lex);
    else if (in.prec == F32)
        hipLaunchKernelGGL(field_unpack_kernel<F32>, grid, dim3(256), 0, s, g, (const char *)in.data, stride,
                           in.parity, scale, (double2 *)lex);
    else
        hipLaunchKernelGGL(field_unpack_kernel<F16>, grid, dim3(256), 0, s, g, (const char *)in.data, stride,
                           in.parity, scale, (double2 *)lex);
    LQS_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------

template <int PI, int PO>
__global__ void convert_kernel(int vh, const char *in, int64_t in_stride, char *out, int64_t out_stride)
{
    typedef typename RealOf<PO>::type TO;
    const int cb = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (cb >= vh) return;
    const auto v = SpinorIO<PI>::load(in + r * in_stride, vh, cb);
    SpinorIO<PO>::store(out + r * out_stride, vh, cb, vcast<TO>(v));
}

template <int PI>
static void convert_from(const Geom &g, int nrhs, const void *in, int prec_out, void *out, hipStream_t s)
{
    dim3 grid((g.vh + 255) / 256, nrhs);
    const int64_t si = field_bytes(g, PI, 1), so = field_bytes(g, prec_out, 1);
    if (prec_out == F64)
        hipLaunchKernelGGL((convert_kernel<PI, F64>), grid, dim3(256), 0, s, g.vh, (const char *)in, si, (char *)out, so);
    else if (prec_out == F32)
        hipLaunchKernelGGL((convert_kernel<PI, F32>), grid, dim3(256), 0, s, g.vh, (const char *)in, si, (char *)out, so);
    else
        hipLaunchKernelGGL((convert_kernel<PI, F16>), grid, dim3(256), 0, s, g.vh, (const char *)in, si, (char *)out, so);
    LQS_HIP(hipGetLastError());
}

void launch_convert(const Geom &g, int nrhs, int prec_in, const void *in, int prec_out, void *out, hipStream_t s)
{
    if (prec_in == F64) convert_from<F64>(g, nrhs, in, prec_out, out, s);
    else if (prec_in == F32) convert_from<F32>(g, nrhs, in, prec_out, out, s);
    else convert_from<F16>(g, nrhs, in, prec_out, out, s);
}

}  // namespace lqs

namespace lqs {

// ---------------------------------------------------------------------------
// sum_sites a^dag b per right-hand side, two fixed-order stages

__global__ void __launch_bounds__(256) field_dot_kernel(int vh, const char *a, const char *b, int64_t stride,
                                                        double *partials, int max_blocks)
{
    const int r = blockIdx.y;
    double re = 0.0, im = 0.0;
    for (int cb = blockIdx.x * blockDim.x + threadIdx.x; cb < vh; cb += gridDim.x * blockDim.x) {
        const V3<double> x = SpinorIO<F64>::load(a + r * stride, vh, cb);
        const V3<double> y = SpinorIO<F64>::load(b + r * stride, vh, cb);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const Cx<double> t = cjmul(x.c[c], y.c[c]);
            re += t.re;
            im += t.im;
        }
    }
    const double sr = block_sum(re);
    const double si = block_sum(im);
    double *pr = partials + (int64_t)r * 2 * max_blocks;
    if (threadIdx.x == 0) {
        pr[blockIdx.x] = sr;
        pr[max_blocks + blockIdx.x] = si;
    }
}

// second stage, one block per right-hand side, fixed order
__global__ void __launch_bounds__(256) field_dot_final(const double *partials, int max_blocks, int nblocks, double *out)
{
    const int r = blockIdx.x;
    const double *pr = partials + (int64_t)r * 2 * max_blocks;
    double re = 0.0, im = 0.0;
    for (int i = threadIdx.x; i < nblocks; i += blockDim.x) {
        re += pr[i];
        im += pr[max_blocks + i];
    }
    const double tr = block_sum(re);
    const double ti = block_sum(im);
    if (threadIdx.x == 0) {
        out[2 * r] = tr;
        out[2 * r + 1] = ti;
    }
}

void launch_field_dot(Ctx &ctx, const Geom &g, int nrhs, const void *a, const void *b, double *out, hipStream_t s)
{
    const int max_blocks = 512;
    int blocks = (int)((g.vh + 255) / 256);
    if (blocks > max_blocks) blocks = max_blocks;
    double *partials = (double *)ctx.workspace("dot.partials", sizeof(double) * 2 * max_blocks * 16);
    hipLaunchKernelGGL(field_dot_kernel, dim3(blocks, nrhs), dim3(256), 0, s, (int)g.vh, (const char *)a,
                       (const char *)b, field_bytes(g, F64, 1), partials, max_blocks);
    LQS_HIP(hipGetLastError());
    hipLaunchKernelGGL(field_dot_final, dim3(nrhs), dim3(256), 0, s, (const double *)partials, max_blocks, blocks, out);
    LQS_HIP(hipGetLastError());
}

}  // namespace lqs

namespace lqs {

// ---------------------------------------------------------------------------
// temporal gauge (Sec. 4.3): a gauge transformation G with G(x, 0) = 1 and
// G(x, t+1) = G(x, t) U_t(x, t) makes U'_t(x) = G(x) U_t(x) G(x + t)^dag = 1
// for t < Nt - 1; U'_mu(x) = G(x) U_mu(x) G(x + mu)^dag for every link.

__device__ __forceinline__ void su3_canonicalise(M3<double> &m)
{
    double n0 = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) n0 += m.e[0][j].re * m.e[0][j].re + m.e[0][j].im * m.e[0][j].im;
    n0 = 1.0 / sqrt(n0);
#pragma unroll
    for (int j = 0; j < 3; ++j) m.e[0][j] = {m.e[0][j].re * n0, m.e[0][j].im * n0};
    Cx<double> d = {0.0, 0.0};
#pragma unroll
    for (int j = 0; j < 3; ++j) d = cadd(d, cjmul(m.e[0][j], m.e[1][j]));
#pragma unroll
    for (int j = 0; j < 3; ++j) m.e[1][j] = csub(m.e[1][j], cmul(d, m.e[0][j]));
    double n1 = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) n1 += m.e[1][j].re * m.e[1][j].re + m.e[1][j].im * m.e[1][j].im;
    n1 = 1.0 / sqrt(n1);
#pragma unroll
    for (int j = 0; j < 3; ++j) m.e[1][j] = {m.e[1][j].re * n1, m.e[1][j].im * n1};
    rebuild_row2(m);
}

__device__ __forceinline__ M3<double> load_canon(const double2 *p)
{
    M3<double> m;
#pragma unroll
    for (int k = 0; k < 9; ++k) m.e[k / 3][k % 3] = {p[k].x, p[k].y};
    return m;
}

__device__ __forceinline__ void store_canon(double2 *p, const M3<double> &m)
{
#pragma unroll
    for (int k = 0; k < 9; ++k) p[k] = make_double2(m.e[k / 3][k % 3].re, m.e[k / 3][k % 3].im);
}

__device__ __forceinline__ M3<double> mm(const M3<double> &a, const M3<double> &b)
{
    M3<double> c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            Cx<double> s = cmul(a.e[i][0], b.e[0][j]);
            s = cadd(s, cmul(a.e[i][1], b.e[1][j]));
            c.e[i][j] = cadd(s, cmul(a.e[i][2], b.e[2][j]));
        }
    return c;
}

// a b^dag
__device__ __forceinline__ M3<double> mmd(const M3<double> &a, const M3<double> &b)
{
    M3<double> c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            Cx<double> s = {0.0, 0.0};
#pragma unroll
            for (int k = 0; k < 3; ++k) s = cadd(s, {a.e[i][k].re * b.e[j][k].re + a.e[i][k].im * b.e[j][k].im,
                                                     a.e[i][k].im * b.e[j][k].re - a.e[i][k].re * b.e[j][k].im});
            c.e[i][j] = s;
        }
    return c;
}

// one thread per spatial site walks the time direction
__global__ void gauge_fix_G_kernel(Geom g, const double2 *U, double2 *G)
{
    const int64_t vs = (int64_t)g.n[0] * g.n[1] * g.n[2];
    const int64_t V = vs * g.n[3];
    const int64_t xs = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (xs >= vs) return;
    M3<double> cur;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) cur.e[i][j] = {i == j ? 1.0 : 0.0, 0.0};
    store_canon(G + 9 * xs, cur);
    for (int t = 0; t + 1 < g.n[3]; ++t) {
        const int64_t lex = xs + vs * t;
        cur = mm(cur, load_canon(U + 9 * (3 * V + lex)));
        su3_canonicalise(cur);
        store_canon(G + 9 * (lex + vs), cur);
    }
}

__global__ void gauge_transform_kernel(Geom g, const double2 *U, const double2 *G, double2 *out)
{
    const int64_t V = 2 * (int64_t)g.vh;
    const int64_t lex = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int mu = blockIdx.y;
    if (lex >= V) return;
    int c[4];
    int64_t r = lex;
    for (int i = 0; i < 4; ++i) {
        c[i] = (int)(r % g.n[i]);
        r /= g.n[i];
    }
    double2 *o = out + 9 * (mu * V + lex);
    if (mu == 3 && c[3] < g.n[3] - 1) {
        M3<double> one;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) one.e[i][j] = {i == j ? 1.0 : 0.0, 0.0};
        store_canon(o, one);
        return;
    }
    c[mu] = (c[mu] + 1) % g.n[mu];
    const int64_t nb = c[0] + (int64_t)g.n[0] * (c[1] + (int64_t)g.n[1] * (c[2] + (int64_t)g.n[2] * c[3]));
    const M3<double> u = mm(load_canon(G + 9 * lex), load_canon(U + 9 * (mu * V + lex)));
    store_canon(o, mmd(u, load_canon(G + 9 * nb)));
}

void launch_gauge_fix_temporal(const Geom &g, const double *links, double *out, double *G, hipStream_t s)
{
    const int64_t vs = (int64_t)g.n[0] * g.n[1] * g.n[2];
    const int64_t V = 2 * (int64_t)g.vh;
    hipLaunchKernelGGL(gauge_fix_G_kernel, dim3((unsigned)((vs + 127) / 128)), dim3(128), 0, s, g,
                       (const double2 *)links, (double2 *)G);
    LQS_HIP(hipGetLastError());
    hipLaunchKernelGGL(gauge_transform_kernel, dim3((unsigned)((V + 255) / 256), 4), dim3(256), 0, s, g,
                       (const double2 *)links, (const double2 *)G, (double2 *)out);
    LQS_HIP(hipGetLastError());
}

// max over t-links with t < Nt - 1 of max |U_ij - delta_ij|, per block
__global__ void __launch_bounds__(256) temporal_violation_kernel(Geom g, const double2 *U, double *partials)
{
    const int64_t V = 2 * (int64_t)g.vh;
    const int64_t vs = V / g.n[3];
    double m = 0.0;
    for (int64_t lex = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; lex < V - vs;
         lex += (int64_t)gridDim.x * blockDim.x) {
        const double2 *u = U + 9 * (3 * V + lex);
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const double re = u[k].x - ((k % 4 == 0) ? 1.0 : 0.0);
            m = fmax(m, fmax(fabs(re), fabs(u[k].y)));
        }
    }
    __shared__ double red[256];
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

double temporal_gauge_violation(Ctx &ctx, const Geom &g, const double *links, hipStream_t s)
{
    const int blocks = 256;
    double *part = (double *)ctx.workspace("tg.partials", sizeof(double) * blocks);
    hipLaunchKernelGGL(temporal_violation_kernel, dim3(blocks), dim3(256), 0, s, g, (const double2 *)links, part);
    LQS_HIP(hipGetLastError());
    std::vector<double> h(blocks);
    LQS_HIP(hipMemcpyAsync(h.data(), part, sizeof(double) * blocks, hipMemcpyDeviceToHost, s));
    LQS_HIP(hipStreamSynchronize(s));
    double m = 0.0;
    for (double v : h) m = v > m ? v : m;  // NaN-free unless the links are
    for (double v : h)
        if (v != v) return v;
    return m;
}

}  // namespace lqs
