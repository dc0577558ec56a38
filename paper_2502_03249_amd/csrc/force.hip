// force.hip -- link derivative of phi^dag M^-1 phi (or of any real function
// of chi = M^-1 phi through its adjoint solve), the "derivatives" a backend
// provides next to the Dirac operator (Sec. 3).  With psi_X = D_oe X:
//   y even: Pi_{y,mu} =  eps_mu(y) [psi_X(y+mu) Y(y)^dag + psi_Y(y+mu) X(y)^dag]
//   y odd : Pi_{y,mu} = -eps_mu(y) [Y(y+mu) psi_X(y)^dag + X(y+mu) psi_Y(y)^dag]
// mode 0 stores F = coeff * (-TA(U Pi)) (su(3)), mode 1 stores coeff * Pi^dag,
// mode 2 adds coeff * (-TA(U Pi)) to out (a momentum update).
// One thread per link; output in the canonical [4][V][3][3] complex layout.
#include "lqs_impl.hpp"

namespace lqs {

__device__ __forceinline__ void outer_add(Cx<double> (&m)[3][3], const V3<double> &a, const V3<double> &b, double s)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            // a_i conj(b_j)
            Cx<double> t = {a.c[i].re * b.c[j].re + a.c[i].im * b.c[j].im, a.c[i].im * b.c[j].re - a.c[i].re * b.c[j].im};
            m[i][j].re += s * t.re;
            m[i][j].im += s * t.im;
        }
}

__global__ void __launch_bounds__(256) force_kernel(Geom g, LinkRef L, const char *X, const char *Y, const char *psx,
                                                    const char *psy, double coeff, int mode, double2 *out)
{
    const int cb = blockIdx.x * blockDim.x + threadIdx.x;
    const int mu = blockIdx.y >> 1, parity = blockIdx.y & 1;
    if (cb >= g.vh) return;
    const Site s = decode(g, cb, parity);
    const double e = ((s.negf >> mu) & 1) ? -1.0 : 1.0;
    const int nb = s.fwd[mu];
    Cx<double> pi[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) pi[i][j] = {0.0, 0.0};
    if (parity == 0) {
        outer_add(pi, SpinorIO<F64>::load(psx, g.vh, nb), SpinorIO<F64>::load(Y, g.vh, cb), e);
        outer_add(pi, SpinorIO<F64>::load(psy, g.vh, nb), SpinorIO<F64>::load(X, g.vh, cb), e);
    } else {
        outer_add(pi, SpinorIO<F64>::load(Y, g.vh, nb), SpinorIO<F64>::load(psx, g.vh, cb), -e);
        outer_add(pi, SpinorIO<F64>::load(X, g.vh, nb), SpinorIO<F64>::load(psy, g.vh, cb), -e);
    }
    double2 *o = out + 9 * ((int64_t)mu * 2 * g.vh + s.lex);
    if (mode == 1) {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) o[3 * i + j] = make_double2(coeff * pi[j][i].re, -coeff * pi[j][i].im);
        return;
    }
    const M3<double> u = LinkIO<F64, 18>::load((const char *)L.base + (2 * mu + parity) * L.block_bytes, g.vh, cb);
    Cx<double> a[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            Cx<double> t = cmul(u.e[i][0], pi[0][j]);
            t = cadd(t, cmul(u.e[i][1], pi[1][j]));
            t = cadd(t, cmul(u.e[i][2], pi[2][j]));
            a[i][j] = t;
        }
    // TA(A) = (A - A^dag)/2 - tr(A - A^dag)/6; F = -coeff * TA(A)
    Cx<double> ta[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) ta[i][j] = {0.5 * (a[i][j].re - a[j][i].re), 0.5 * (a[i][j].im + a[j][i].im)};
    const double tri = (ta[0][0].im + ta[1][1].im + ta[2][2].im) / 3.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) ta[i][i].im -= tri;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double2 r = make_double2(-coeff * ta[i][j].re, -coeff * ta[i][j].im);
            if (mode == 2) {
                const double2 p = o[3 * i + j];
                r.x += p.x;
                r.y += p.y;
            }
            o[3 * i + j] = r;
        }
}

void launch_force(const Geom &g, LinkRef links64, const double *X, const double *Y, const double *psx,
                  const double *psy, double coeff, int mode, double *out, hipStream_t s)
{
    dim3 grid((g.vh + 255) / 256, 8);
    hipLaunchKernelGGL(force_kernel, grid, dim3(256), 0, s, g, links64, (const char *)X, (const char *)Y,
                       (const char *)psx, (const char *)psy, coeff, mode, (double2 *)out);
    LQS_HIP(hipGetLastError());
}

}  // namespace lqs
