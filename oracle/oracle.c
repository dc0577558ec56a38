/*
 * oracle.c -- plain FP64 CPU reference for the staggered even-odd solver.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this file.  It shares no code, header,
 * table or constant with the GPU library and neither side includes the other.
 *
 * What it computes (Kumar, Borsanyi, Guenther, Wong, "Portable Lattice QCD
 * implementation based on OpenCL", LATTICE2024):
 *   - the staggered operator of eq. (1) (Sec. 4.2) on the full lattice,
 *   - its restriction to one output parity (the "hop" D_eo or D_oe),
 *   - its adjoint, written as the conjugate transpose of the stencil,
 *   - the even-odd normal operator M = m^2 - D_eo D_oe,
 *   - conjugate gradient on M (the inversion of Sec. 4.2),
 *   - the derivative of phi^dag M^-1 phi with respect to the links (the
 *     "derivatives" a backend provides, Sec. 3), from dS = -chi^dag dM chi.
 *
 * Conventions where the paper is silent (each is a reading, not a citation):
 *   - direction mu = 0,1,2,3 is x,y,z,t; lex = x + Nx (y + Ny (z + Nz t));
 *   - eta_0 = 1, eta_1 = (-1)^x, eta_2 = (-1)^(x+y), eta_3 = (-1)^(x+y+z);
 *   - periodic in x,y,z, antiperiodic in t: the phase of the t-link leaving a
 *     site with t = Nt-1 carries an extra -1;
 *   - in eq. (1) the phase in the backward term is the phase of the link
 *     (x - mu, mu) itself, boundary sign included;
 *   - eq. (1) is taken literally, without a factor 1/2;
 *   - a site is even when x+y+z+t is even.
 *
 * Storage: complex numbers are (re, im) doubles.  Links [4][V][3][3] with
 * row-major 3x3 blocks; colour vectors [V][3], lexicographic sites.  Fields of
 * one parity are stored on the full lattice with zeros on the other parity.
 * All extents must be even.  Built with -ffp-contract=off; reductions are
 * serial in site order.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

typedef struct {
    int n[4];
    long vol;
} geom;

static geom make_geom(const int32_t dims[4])
{
    geom g;
    for (int i = 0; i < 4; ++i) g.n[i] = dims[i];
    g.vol = (long)dims[0] * dims[1] * dims[2] * dims[3];
    return g;
}

static void coords(const geom *g, long lex, int c[4])
{
    for (int i = 0; i < 4; ++i) {
        c[i] = (int)(lex % g->n[i]);
        lex /= g->n[i];
    }
}

static long lexof(const geom *g, const int c[4])
{
    return c[0] + (long)g->n[0] * (c[1] + (long)g->n[1] * (c[2] + (long)g->n[2] * c[3]));
}

/* Site x + step * mu-hat, periodic wrap (the boundary sign lives in the phase). */
static long shift(const geom *g, long lex, int mu, int step)
{
    int c[4];
    coords(g, lex, c);
    c[mu] = (c[mu] + step + g->n[mu]) % g->n[mu];
    return lexof(g, c);
}

static int site_parity(const geom *g, long lex)
{
    int c[4];
    coords(g, lex, c);
    return (c[0] + c[1] + c[2] + c[3]) & 1;
}

/* Kogut-Susskind phase eta_mu at coordinates c. */
static double eta(int mu, const int c[4])
{
    int s = 0;
    for (int nu = 0; nu < mu; ++nu) s += c[nu];
    return (s & 1) ? -1.0 : 1.0;
}

/* Phase of the link (x, mu): eta_mu(x), times -1 for a t-link leaving t = Nt-1. */
static double link_phase(const geom *g, long lex, int mu)
{
    int c[4];
    coords(g, lex, c);
    double e = eta(mu, c);
    if (mu == 3 && c[3] == g->n[3] - 1) e = -e;
    return e;
}

static const cplx *link(const cplx *u, const geom *g, int mu, long lex)
{
    return u + 9 * ((long)mu * g->vol + lex);
}

/* y += s * U v */
static void add_mv(cplx y[3], double s, const cplx *u, const cplx *v)
{
    for (int a = 0; a < 3; ++a) {
        cplx t = 0.0;
        for (int b = 0; b < 3; ++b) t += u[3 * a + b] * v[b];
        y[a] += s * t;
    }
}

/* y += s * U^dag v */
static void add_mdv(cplx y[3], double s, const cplx *u, const cplx *v)
{
    for (int a = 0; a < 3; ++a) {
        cplx t = 0.0;
        for (int b = 0; b < 3; ++b) t += conj(u[3 * b + a]) * v[b];
        y[a] += s * t;
    }
}

/* Eq. (1) at one site x. */
static void dslash_site(const geom *g, const cplx *u, const cplx *in, long x, cplx out[3])
{
    out[0] = out[1] = out[2] = 0.0;
    for (int mu = 0; mu < 4; ++mu) {
        long xf = shift(g, x, mu, +1);
        long xb = shift(g, x, mu, -1);
        add_mv(out, link_phase(g, x, mu), link(u, g, mu, x), in + 3 * xf);
        add_mdv(out, -link_phase(g, xb, mu), link(u, g, mu, xb), in + 3 * xb);
    }
}

/*
 * out = D in.  out_parity -1: every site.  0 or 1: only sites of that parity
 * are computed (the hop D_{p,1-p}; their neighbours all have parity 1-p), the
 * other sites of out are set to zero.
 */
void ora_dslash(const int32_t dims[4], const double *U, const double *in, double *out, int32_t out_parity)
{
    geom g = make_geom(dims);
    const cplx *u = (const cplx *)U;
    const cplx *v = (const cplx *)in;
    cplx *w = (cplx *)out;
#pragma omp parallel for schedule(static)
    for (long x = 0; x < g.vol; ++x) {
        if (out_parity >= 0 && site_parity(&g, x) != out_parity) {
            w[3 * x] = w[3 * x + 1] = w[3 * x + 2] = 0.0;
            continue;
        }
        dslash_site(&g, u, v, x, w + 3 * x);
    }
}

/*
 * out = D^dag in, computed as the conjugate transpose of the stencil: every
 * block D_{y,x} of row y is scattered as (D_{y,x})^dag in_y into out_x.  The
 * row y contains D_{y,y+mu} = eps_mu(y) U_{y,mu} and
 * D_{y,y-mu} = -eps_mu(y-mu) U^dag_{y-mu,mu}.  Serial (scatter).
 * out_parity selects which output sites are kept (others zeroed), as above.
 */
void ora_dslash_dagger(const int32_t dims[4], const double *U, const double *in, double *out, int32_t out_parity)
{
    geom g = make_geom(dims);
    const cplx *u = (const cplx *)U;
    const cplx *v = (const cplx *)in;
    cplx *w = (cplx *)out;
    memset(w, 0, sizeof(cplx) * 3 * g.vol);
    for (long y = 0; y < g.vol; ++y) {
        for (int mu = 0; mu < 4; ++mu) {
            long yf = shift(&g, y, mu, +1);
            long yb = shift(&g, y, mu, -1);
            /* (eps U_{y,mu})^dag in_y  ->  out_{y+mu} */
            add_mdv(w + 3 * yf, link_phase(&g, y, mu), link(u, &g, mu, y), v + 3 * y);
            /* (-eps U^dag_{y-mu,mu})^dag in_y = -eps U_{y-mu,mu} in_y  ->  out_{y-mu} */
            add_mv(w + 3 * yb, -link_phase(&g, yb, mu), link(u, &g, mu, yb), v + 3 * y);
        }
    }
    if (out_parity >= 0)
        for (long x = 0; x < g.vol; ++x)
            if (site_parity(&g, x) != out_parity) w[3 * x] = w[3 * x + 1] = w[3 * x + 2] = 0.0;
}

/* out = M in = m^2 in - D_eo D_oe in on even sites (odd sites of in ignored, of out zero). */
void ora_normal(const int32_t dims[4], const double *U, double mass, const double *in, double *out)
{
    geom g = make_geom(dims);
    cplx *even = malloc(sizeof(cplx) * 3 * g.vol);
    cplx *odd = malloc(sizeof(cplx) * 3 * g.vol);
    const cplx *v = (const cplx *)in;
    cplx *w = (cplx *)out;
    for (long x = 0; x < g.vol; ++x)
        for (int c = 0; c < 3; ++c) even[3 * x + c] = site_parity(&g, x) == 0 ? v[3 * x + c] : 0.0;
    ora_dslash(dims, U, (const double *)even, (double *)odd, 1);  /* D_oe */
    ora_dslash(dims, U, (const double *)odd, out, 0);             /* D_eo */
    for (long x = 0; x < g.vol; ++x)
        for (int c = 0; c < 3; ++c) w[3 * x + c] = mass * mass * even[3 * x + c] - w[3 * x + c];
    free(even);
    free(odd);
}

static double norm2(const cplx *a, long n)
{
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += creal(a[i]) * creal(a[i]) + cimag(a[i]) * cimag(a[i]);
    return s;
}

static double re_dot(const cplx *a, const cplx *b, long n)
{
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += creal(conj(a[i]) * b[i]);
    return s;
}

/* ||b - M x|| / ||b|| on even sites. */
double ora_true_residual(const int32_t dims[4], const double *U, double mass, const double *b, const double *x)
{
    geom g = make_geom(dims);
    long n = 3 * g.vol;
    cplx *mx = malloc(sizeof(cplx) * n);
    ora_normal(dims, U, mass, x, (double *)mx);
    const cplx *bb = (const cplx *)b;
    double r2 = 0.0, b2 = 0.0;
    for (long x0 = 0; x0 < g.vol; ++x0) {
        if (site_parity(&g, x0) != 0) continue;
        for (int c = 0; c < 3; ++c) {
            cplx d = bb[3 * x0 + c] - mx[3 * x0 + c];
            r2 += creal(d) * creal(d) + cimag(d) * cimag(d);
            b2 += creal(bb[3 * x0 + c]) * creal(bb[3 * x0 + c]) + cimag(bb[3 * x0 + c]) * cimag(bb[3 * x0 + c]);
        }
    }
    free(mx);
    return sqrt(r2) / sqrt(b2);
}

/*
 * Conjugate gradient (Hestenes-Stiefel) for M x = b on even sites.
 * x holds the starting guess on entry (zero for a cold start) and the
 * solution on exit.  Iterates until ||r|| <= tol ||b|| for the recursively
 * updated residual, then recomputes r = b - M x; if that true residual
 * exceeds tol the iteration restarts from x (p = r).  Returns 0 on success,
 * 1 if max_iter iterations did not suffice, -1 on breakdown (p.Mp <= 0 or
 * non-finite).  iters receives the number of applications of M inside the
 * iteration, true_res the final ||b - Mx|| / ||b||.
 */
int32_t ora_cg(const int32_t dims[4], const double *U, double mass, const double *b, double *x,
               double tol, int32_t max_iter, int32_t *iters, double *true_res)
{
    geom g = make_geom(dims);
    long n = 3 * g.vol;
    cplx *r = malloc(sizeof(cplx) * n);
    cplx *p = malloc(sizeof(cplx) * n);
    cplx *q = malloc(sizeof(cplx) * n);
    cplx *xx = (cplx *)x;
    const cplx *bb = (const cplx *)b;
    int32_t status = 1;
    int32_t k = 0;
    double b2 = norm2(bb, n);

    ora_normal(dims, U, mass, x, (double *)q);
    for (long i = 0; i < n; ++i) r[i] = bb[i] - q[i];
    memcpy(p, r, sizeof(cplx) * n);
    double rho = norm2(r, n);

    while (k < max_iter) {
        if (rho <= tol * tol * b2) {
            ora_normal(dims, U, mass, x, (double *)q);
            for (long i = 0; i < n; ++i) r[i] = bb[i] - q[i];
            rho = norm2(r, n);
            if (rho <= tol * tol * b2) { status = 0; break; }
            memcpy(p, r, sizeof(cplx) * n);
        }
        ora_normal(dims, U, mass, (const double *)p, (double *)q);
        ++k;
        double pq = re_dot(p, q, n);
        if (!(pq > 0.0) || !isfinite(pq)) { status = -1; break; }
        double alpha = rho / pq;
        for (long i = 0; i < n; ++i) {
            xx[i] += alpha * p[i];
            r[i] -= alpha * q[i];
        }
        double rho_new = norm2(r, n);
        double beta = rho_new / rho;
        for (long i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
        rho = rho_new;
    }
    double tr = ora_true_residual(dims, U, mass, b, x);
    if (status != -1) status = (tr <= tol) ? 0 : 1;
    if (iters) *iters = k;
    if (true_res) *true_res = tr;
    free(r);
    free(p);
    free(q);
    return status;
}

/* Traceless anti-Hermitian part: TA(A) = (A - A^dag)/2 - tr(A - A^dag)/6 * 1. */
static void traceless_antiherm(const cplx a[9], cplx out[9])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) out[3 * i + j] = 0.5 * (a[3 * i + j] - conj(a[3 * j + i]));
    cplx tr = (out[0] + out[4] + out[8]) / 3.0;
    out[0] -= tr;
    out[4] -= tr;
    out[8] -= tr;
}

/*
 * Link derivative of a real function L(chi) of chi = M^-1 phi, given
 * X = chi and Y = M^-1 g (g = 2 dL/dchi^*); for L = phi^dag M^-1 phi both are
 * chi.  From dL = Re( Y^dag dD_eo D_oe X - (D_oe Y)^dag dD_oe X ) one finds
 * dL = Re sum_links tr(dU_{y,mu} Pi_{y,mu}) with, writing psi_X = D_oe X,
 *   y even: Pi = eps_mu(y) [ psi_X(y+mu) Y(y)^dag + psi_Y(y+mu) X(y)^dag ]
 *   y odd : Pi = -eps_mu(y) [ Y(y+mu) psi_X(y)^dag + X(y+mu) psi_Y(y)^dag ]
 * mode 0 writes F = coeff * (-TA(U Pi)), the su(3) element with
 *   dL/dw = Re tr(F^dag A) for U -> exp(w A) U, A in su(3);
 * mode 1 writes coeff * Pi^dag, the gradient with respect to the real and
 * imaginary parts of every link entry (grad = dL/dRe + i dL/dIm).
 * Y == NULL means Y = X.  X, Y: even-site fields.  F: [4][V][3][3].
 */
void ora_force(const int32_t dims[4], const double *U, const double *X, const double *Y, double coeff,
               int32_t mode, double *F)
{
    geom g = make_geom(dims);
    long n = 3 * g.vol;
    const cplx *u = (const cplx *)U;
    const cplx *xf = (const cplx *)X;
    const cplx *yf = (const cplx *)(Y ? Y : X);
    cplx *psx = malloc(sizeof(cplx) * n);
    cplx *psy = malloc(sizeof(cplx) * n);
    cplx *out = (cplx *)F;
    ora_dslash(dims, U, X, (double *)psx, 1);
    ora_dslash(dims, U, (const double *)yf, (double *)psy, 1);
    for (int mu = 0; mu < 4; ++mu) {
        for (long y = 0; y < g.vol; ++y) {
            long yf1 = shift(&g, y, mu, +1);
            double e = link_phase(&g, y, mu);
            cplx pi[9];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    if (site_parity(&g, y) == 0)
                        pi[3 * a + b] = e * (psx[3 * yf1 + a] * conj(yf[3 * y + b]) +
                                             psy[3 * yf1 + a] * conj(xf[3 * y + b]));
                    else
                        pi[3 * a + b] = -e * (yf[3 * yf1 + a] * conj(psx[3 * y + b]) +
                                              xf[3 * yf1 + a] * conj(psy[3 * y + b]));
                }
            cplx *o = out + 9 * ((long)mu * g.vol + y);
            if (mode == 1) {
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) o[3 * a + b] = coeff * conj(pi[3 * b + a]);
            } else {
                const cplx *um = link(u, &g, mu, y);
                cplx upi[9], ta[9];
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) {
                        cplx s = 0.0;
                        for (int k = 0; k < 3; ++k) s += um[3 * a + k] * pi[3 * k + b];
                        upi[3 * a + b] = s;
                    }
                traceless_antiherm(upi, ta);
                for (int i = 0; i < 9; ++i) o[i] = -coeff * ta[i];
            }
        }
    }
    free(psx);
    free(psy);
}

/* Threads for the oracle's parallel regions (n >= 1; no effect without OpenMP). */
void ora_set_threads(int32_t n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Number of OpenMP threads a parallel region of the oracle uses (1 without OpenMP). */
int32_t ora_threads(void)
{
    int32_t t = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            t = (int32_t)omp_get_num_threads();
#endif
        }
    }
    return t;
}
