// force.hip -- link derivative of phi^dag M^-1 phi (or of any real function
// of chi = M^-1 phi through its adjoint solve), the "derivatives" a backend
// provides next to the Dirac operator (Sec. 3).  With psi_X = D_oe X:
//   y even: Pi_{y,mu} =  eps_mu(y) [psi_X(y+mu) Y(y)^dag + psi_Y(y+mu) X(y)^dag]
//   y odd : Pi_{y,mu} = -eps_mu(y) [Y(y+mu) psi_X(y)^dag + X(y+mu) psi_Y(y)^dag]
// mode 0 stores F = coeff * (-TA(U Pi)) (su(3)), mode 1 stores coeff * Pi^dag,
// mode 2 adds coeff * (-TA(U Pi)) to out (a momentum update).
// Output in the canonical [4][V][3][3] complex layout.
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

// One thread per link (mu, x) in lexicographic site order, so that a wave
// writes 64 consecutive 144-byte output records (a parity-split grid left
// every other record to another block and halved the write efficiency).
// The two parities use the same code with their operands selected by address.
__global__ void __launch_bounds__(256) force_kernel(Geom g, LinkRef L, const char *X, const char *Y, const char *psx,
                                                    const char *psy, double coeff, int mode, double2 *out)
{
    const int lex = blockIdx.x * blockDim.x + threadIdx.x;
    const int mu = blockIdx.y;
    if (lex >= 2 * g.vh) return;
    int q = lex / g.n[0];
    const int xc = lex - q * g.n[0];
    const int y = q % g.n[1];
    q /= g.n[1];
    const int parity = (xc + y + q % g.n[2] + q / g.n[2]) & 1;
    const int cb = lex >> 1;
    const Site s = decode(g, cb, parity);
    const double e = ((s.negf >> mu) & 1) ? -1.0 : 1.0;
    const int nb = s.fwd[mu];
    // y even: Pi = e [psi_X(y+mu) Y(y)^dag + psi_Y(y+mu) X(y)^dag]
    // y odd : Pi = -e [Y(y+mu) psi_X(y)^dag + X(y+mu) psi_Y(y)^dag]
    const bool ev = parity == 0;
    const char *a1 = ev ? psx : Y, *b1 = ev ? Y : psx, *a2 = ev ? psy : X, *b2 = ev ? X : psy;
    Cx<double> pi[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) pi[i][j] = {0.0, 0.0};
    outer_add(pi, SpinorIO<F64>::load(a1, g.vh, nb), SpinorIO<F64>::load(b1, g.vh, cb), ev ? e : -e);
    outer_add(pi, SpinorIO<F64>::load(a2, g.vh, nb), SpinorIO<F64>::load(b2, g.vh, cb), ev ? e : -e);
    double2 *o = out + 9 * ((int64_t)mu * 2 * g.vh + lex);
    // accumulate mode: fetch the old record up front, so that its loads overlap
    // the arithmetic instead of alternating with the stores
    double2 prev[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) prev[k] = mode == 2 ? o[k] : make_double2(0.0, 0.0);
    if (mode == 1) {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) o[3 * i + j] = make_double2(coeff * pi[j][i].re, -coeff * pi[j][i].im);
        return;
    }
    const M3<double> u = LinkIO<F64, 18>::load((const char *)L.base + (2 * mu + parity) * L.block_bytes, L.pitch, cb);
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
            o[3 * i + j] = make_double2(prev[3 * i + j].x - coeff * ta[i][j].re, prev[3 * i + j].y - coeff * ta[i][j].im);
        }
}

void launch_force(const Geom &g, LinkRef links64, const double *X, const double *Y, const double *psx,
                  const double *psy, double coeff, int mode, double *out, hipStream_t s)
{
    dim3 grid((2 * g.vh + 255) / 256, 4);
    hipLaunchKernelGGL(force_kernel, grid, dim3(256), 0, s, g, links64, (const char *)X, (const char *)Y,
                       (const char *)psx, (const char *)psy, coeff, mode, (double2 *)out);
    LQS_HIP(hipGetLastError());
}

}  // namespace lqs
