/*
 * hmc.c -- plain FP64 CPU reference for hybrid Monte Carlo with staggered
 * fermions: the Wilson plaquette action and its link derivative, the SU(3)
 * exponential, the pseudofermion heat bath and one molecular-dynamics
 * trajectory with a Metropolis decision.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite and the benchmark's CPU
 * baseline load this file.  It shares no code, header, table or constant with
 * the GPU library.  It calls the staggered operator, CG and fermion
 * derivative of oracle.c (same shared object).
 *
 * The paper names HMC, the gauge action and its derivatives as the
 * simulation layer its backends serve (Sec. 3) and the inversion as the
 * dominant cost inside it (Sec. 1); it gives none of the formulas below, so
 * each is the textbook definition, written out with the conventions stated
 * here.
 *
 *   Plaquette action:  S_g = beta * sum_x sum_{mu<nu} (1 - Re tr P_{mu nu}(x) / 3),
 *     P_{mu nu}(x) = U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag, links periodic
 *     in every direction (the antiperiodic sign belongs to the fermions only).
 *   Momenta: Q on every link, anti-Hermitian traceless, Q = sum_a q_a T_a with
 *     T_a = i lambda_a / 2 (Gell-Mann lambda); kinetic energy
 *     K = -sum_links tr(Q^2) = 1/2 sum q_a^2, so q_a ~ N(0,1) is the heat bath.
 *   Force convention: for a function S of the links, F is the su(3) element
 *     with dS/dw = Re tr(F^dag A) for U -> exp(w A) U, A in su(3).  Then
 *     dq_a/dtau = -dS/dw_a = -f_a / 2, i.e. dQ/dtau = -F/2, dU/dtau = Q U.
 *     Gauge part: F_g = (beta/3) TA(U V), V the sum of the six staples of the
 *     link; fermion part: F_f = -TA(U Pi) from ora_force with X = Y = chi.
 *   Pseudofermion: phi = m eta_e - D_eo eta_o, eta complex Gaussian on every
 *     site with density ~ exp(-eta^dag eta); then <phi phi^dag> = M and
 *     S_f = phi^dag M^-1 phi with M = m^2 - D_eo D_oe (even sites).
 *   H = K + S_g + S_f (S_f dropped when fermions are off).
 *   Integrators over n steps of h = tau / n:
 *     leapfrog: Q -= h/2 G; then n times { U = exp(h Q) U; Q -= h G }, the last
 *       momentum step being h/2;
 *     Omelyan (second-order minimum-norm, parameter lam): per step
 *       Q -= lam h G; U = exp(h/2 Q) U; Q -= (1 - 2 lam) h G; U = exp(h/2 Q) U;
 *       Q -= lam h G;
 *     with G = F/2 evaluated on the current links.
 *   Metropolis: accept when u < exp(-(H1 - H0)), u uniform in [0,1) given.
 *
 * Storage as in oracle.c: links and momenta [4][V][3][3] complex (re, im)
 * doubles, colour vectors [V][3], lexicographic sites.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* from oracle.c */
void ora_dslash(const int32_t dims[4], const double *U, const double *in, double *out, int32_t out_parity);
int32_t ora_cg(const int32_t dims[4], const double *U, double mass, const double *b, double *x, double tol,
               int32_t max_iter, int32_t *iters, double *true_res);
void ora_force(const int32_t dims[4], const double *U, const double *X, const double *Y, double coeff,
               int32_t mode, double *F);

typedef struct {
    int n[4];
    long vol;
} hgeom;

static hgeom hmake(const int32_t dims[4])
{
    hgeom g;
    for (int i = 0; i < 4; ++i) g.n[i] = dims[i];
    g.vol = (long)dims[0] * dims[1] * dims[2] * dims[3];
    return g;
}

static long hshift(const hgeom *g, long lex, int mu, int step)
{
    int c[4];
    long l = lex;
    for (int i = 0; i < 4; ++i) {
        c[i] = (int)(l % g->n[i]);
        l /= g->n[i];
    }
    c[mu] = (c[mu] + step + g->n[mu]) % g->n[mu];
    return c[0] + (long)g->n[0] * (c[1] + (long)g->n[1] * (c[2] + (long)g->n[2] * c[3]));
}

static int hparity(const hgeom *g, long lex)
{
    int s = 0;
    for (int i = 0; i < 4; ++i) {
        s += (int)(lex % g->n[i]);
        lex /= g->n[i];
    }
    return s & 1;
}

/* 3x3 complex helpers, row-major */
static void mm(const cplx *a, const cplx *b, cplx *c)
{
    cplx t[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx s = 0.0;
            for (int k = 0; k < 3; ++k) s += a[3 * i + k] * b[3 * k + j];
            t[3 * i + j] = s;
        }
    memcpy(c, t, sizeof(t));
}

static void dag(const cplx *a, cplx *c)
{
    cplx t[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) t[3 * i + j] = conj(a[3 * j + i]);
    memcpy(c, t, sizeof(t));
}

static const cplx *lk(const cplx *u, const hgeom *g, int mu, long x) { return u + 9 * ((long)mu * g->vol + x); }

/*
 * exp(A) for a 3x3 complex matrix: scaling and squaring of the Taylor
 * series.  A is divided by 2^s so that its max-row-sum norm is at most 1/2,
 * the series is summed to 24 terms (remainder below 1e-30 relative), and the
 * result squared s times.
 */
void ora_expm3(const double *A, double *out)
{
    const cplx *a = (const cplx *)A;
    double nrm = 0.0;
    for (int i = 0; i < 3; ++i) {
        double r = 0.0;
        for (int j = 0; j < 3; ++j) r += cabs(a[3 * i + j]);
        if (r > nrm) nrm = r;
    }
    int s = 0;
    while (nrm > 0.5) {
        nrm *= 0.5;
        ++s;
    }
    double sc = ldexp(1.0, -s);
    cplx b[9], term[9], sum[9];
    for (int i = 0; i < 9; ++i) {
        b[i] = a[i] * sc;
        term[i] = (i % 4 == 0) ? 1.0 : 0.0;
        sum[i] = term[i];
    }
    for (int k = 1; k <= 24; ++k) {
        mm(term, b, term);
        for (int i = 0; i < 9; ++i) {
            term[i] /= (double)k;
            sum[i] += term[i];
        }
    }
    for (int k = 0; k < s; ++k) mm(sum, sum, sum);
    memcpy(out, sum, sizeof(sum));
}

/* The plaquette P_{mu nu}(x). */
static void plaquette(const hgeom *g, const cplx *u, long x, int mu, int nu, cplx *p)
{
    cplx t[9], d[9];
    long xm = hshift(g, x, mu, 1), xn = hshift(g, x, nu, 1);
    mm(lk(u, g, mu, x), lk(u, g, nu, xm), t);
    dag(lk(u, g, mu, xn), d);
    mm(t, d, t);
    dag(lk(u, g, nu, x), d);
    mm(t, d, p);
}

/* S_g = beta * sum_x sum_{mu<nu} (1 - Re tr P / 3), summed serially in site order. */
double ora_plaquette_action(const int32_t dims[4], const double *U, double beta)
{
    hgeom g = hmake(dims);
    const cplx *u = (const cplx *)U;
    double s = 0.0;
    for (long x = 0; x < g.vol; ++x)
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu) {
                cplx p[9];
                plaquette(&g, u, x, mu, nu, p);
                s += 1.0 - creal(p[0] + p[4] + p[8]) / 3.0;
            }
    return beta * s;
}

/* Sum of the six staples V of link (x, mu): Re tr(U_mu(x) V) collects every
 * plaquette that contains the link. */
static void staples(const hgeom *g, const cplx *u, long x, int mu, cplx *v)
{
    for (int i = 0; i < 9; ++i) v[i] = 0.0;
    long xm = hshift(g, x, mu, 1);
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        cplx t[9], d[9];
        /* upper: U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag */
        long xn = hshift(g, x, nu, 1);
        dag(lk(u, g, mu, xn), d);
        mm(lk(u, g, nu, xm), d, t);
        dag(lk(u, g, nu, x), d);
        mm(t, d, t);
        for (int i = 0; i < 9; ++i) v[i] += t[i];
        /* lower: U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu) */
        long xdn = hshift(g, x, nu, -1), xmdn = hshift(g, xm, nu, -1);
        dag(lk(u, g, nu, xmdn), t);
        dag(lk(u, g, mu, xdn), d);
        mm(t, d, t);
        mm(t, lk(u, g, nu, xdn), t);
        for (int i = 0; i < 9; ++i) v[i] += t[i];
    }
}

static void ta(const cplx *a, cplx *out)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) out[3 * i + j] = 0.5 * (a[3 * i + j] - conj(a[3 * j + i]));
    cplx tr = (out[0] + out[4] + out[8]) / 3.0;
    out[0] -= tr;
    out[4] -= tr;
    out[8] -= tr;
}

/* F_g = coeff * (beta/3) TA(U V) on every link (overwrites F). */
void ora_gauge_force(const int32_t dims[4], const double *U, double beta, double coeff, double *F)
{
    hgeom g = hmake(dims);
    const cplx *u = (const cplx *)U;
    cplx *f = (cplx *)F;
    for (int mu = 0; mu < 4; ++mu)
        for (long x = 0; x < g.vol; ++x) {
            cplx v[9], w[9], t[9];
            staples(&g, u, x, mu, v);
            mm(lk(u, &g, mu, x), v, w);
            ta(w, t);
            cplx *o = f + 9 * ((long)mu * g.vol + x);
            for (int i = 0; i < 9; ++i) o[i] = coeff * (beta / 3.0) * t[i];
        }
}

/* K = -sum_links tr(Q^2). */
double ora_kinetic(const int32_t dims[4], const double *Q)
{
    hgeom g = hmake(dims);
    const cplx *q = (const cplx *)Q;
    double k = 0.0;
    for (long l = 0; l < 4 * g.vol; ++l) {
        const cplx *m = q + 9 * l;
        cplx tr = 0.0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) tr += m[3 * i + j] * m[3 * j + i];
        k -= creal(tr);
    }
    return k;
}

/* phi = m eta_e - D_eo eta_o on even sites, zero on odd sites. */
void ora_pseudofermion(const int32_t dims[4], const double *U, double mass, const double *eta, double *phi)
{
    hgeom g = hmake(dims);
    long n = 3 * g.vol;
    const cplx *e = (const cplx *)eta;
    cplx *p = (cplx *)phi;
    cplx *d = malloc(sizeof(cplx) * n);
    ora_dslash(dims, U, eta, (double *)d, 0);
    for (long x = 0; x < g.vol; ++x)
        for (int a = 0; a < 3; ++a)
            p[3 * x + a] = hparity(&g, x) == 0 ? mass * e[3 * x + a] - d[3 * x + a] : 0.0;
    free(d);
}

typedef struct {
    const int32_t *dims;
    hgeom g;
    double beta, mass, tol;
    int fermions;
    const double *phi;
    double *chi;     /* current M^-1 phi (even sites) */
    int32_t iters;   /* CG iterations so far */
    int32_t solves;
    int32_t fail;
} md_ctx;

/* chi = M^-1 phi on the links U (CG from zero); S_f = Re phi^dag chi. */
static double fermion_solve(md_ctx *c, const double *U)
{
    long n = 3 * c->g.vol;
    memset(c->chi, 0, sizeof(cplx) * n);
    int32_t it = 0;
    double tr = 0.0;
    int32_t st = ora_cg(c->dims, U, c->mass, c->phi, c->chi, c->tol, 100000, &it, &tr);
    if (st != 0) c->fail = 1;
    c->iters += it;
    c->solves += 1;
    const cplx *p = (const cplx *)c->phi, *x = (const cplx *)c->chi;
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += creal(conj(p[i]) * x[i]);
    return s;
}

/* Q -= eps * G(U), G = (F_g + F_f) / 2. */
static void momentum_step(md_ctx *c, const double *U, double *Q, double eps)
{
    long nl = 9 * 4 * c->g.vol;
    double *f = malloc(sizeof(cplx) * nl);
    cplx *q = (cplx *)Q;
    const cplx *ff = (const cplx *)f;
    ora_gauge_force(c->dims, U, c->beta, 1.0, f);
    for (long i = 0; i < nl; ++i) q[i] -= 0.5 * eps * ff[i];
    if (c->fermions) {
        fermion_solve(c, U);
        ora_force(c->dims, U, c->chi, NULL, 1.0, 0, f);
        for (long i = 0; i < nl; ++i) q[i] -= 0.5 * eps * ff[i];
    }
    free(f);
}

/* U = exp(eps Q) U on every link. */
static void link_step(const hgeom *g, double *U, const double *Q, double eps)
{
    cplx *u = (cplx *)U;
    const cplx *q = (const cplx *)Q;
    for (long l = 0; l < 4 * g->vol; ++l) {
        cplx a[9], e[9];
        for (int i = 0; i < 9; ++i) a[i] = eps * q[9 * l + i];
        ora_expm3((const double *)a, (double *)e);
        mm(e, u + 9 * l, u + 9 * l);
    }
}

/* U = exp(eps Q) U on every link (exported for the parity tests). */
void ora_link_update(const int32_t dims[4], double *U, const double *Q, double eps)
{
    hgeom g = hmake(dims);
    link_step(&g, U, Q, eps);
}

/*
 * One trajectory.  In: U0 (links), Q0 (momenta), pf (fermions = 1: the
 * heat-bath Gaussians eta, from which phi is made on U0; fermions = 2: phi
 * itself, e.g. to run a trajectory backwards; ignored when fermions = 0), u
 * (uniform in [0,1)).  Out: U1, Q1 (the proposal at the end of the
 * trajectory), energies[6] = {K0, Sg0, Sf0, K1, Sg1, Sf1}, *accepted,
 * *cg_iters (all CG iterations), *cg_solves, and phi_out (if not NULL) the
 * pseudofermion used.  integrator 0: leapfrog; 1: Omelyan with parameter
 * lam.  Returns 0, or 1 if a CG did not reach tol.
 */
int32_t ora_hmc(const int32_t dims[4], const double *U0, const double *Q0, const double *pf, double mass,
                double beta, double tau, int32_t nsteps, int32_t integrator, double lam, int32_t fermions,
                double cg_tol, double u, double *U1, double *Q1, double *energies, int32_t *accepted,
                int32_t *cg_iters, int32_t *cg_solves, double *phi_out)
{
    md_ctx c;
    c.dims = dims;
    c.g = hmake(dims);
    c.beta = beta;
    c.mass = mass;
    c.tol = cg_tol;
    c.fermions = fermions;
    c.iters = 0;
    c.solves = 0;
    c.fail = 0;
    long n = 3 * c.g.vol, nl = 9 * 4 * c.g.vol;
    double *phi = calloc(n, sizeof(cplx));
    c.chi = calloc(n, sizeof(cplx));
    c.phi = phi;
    memcpy(U1, U0, sizeof(cplx) * nl);
    memcpy(Q1, Q0, sizeof(cplx) * nl);

    double sf0 = 0.0, sf1 = 0.0;
    if (fermions == 1) ora_pseudofermion(dims, U0, mass, pf, phi);
    else if (fermions == 2) memcpy(phi, pf, sizeof(cplx) * n);
    if (fermions) sf0 = fermion_solve(&c, U0);
    if (phi_out) memcpy(phi_out, phi, sizeof(cplx) * n);
    double k0 = ora_kinetic(dims, Q0), sg0 = ora_plaquette_action(dims, U0, beta);

    const double h = tau / nsteps;
    if (integrator == 0) {
        momentum_step(&c, U1, Q1, 0.5 * h);
        for (int s = 0; s < nsteps; ++s) {
            link_step(&c.g, U1, Q1, h);
            momentum_step(&c, U1, Q1, s == nsteps - 1 ? 0.5 * h : h);
        }
    } else {
        for (int s = 0; s < nsteps; ++s) {
            momentum_step(&c, U1, Q1, lam * h);
            link_step(&c.g, U1, Q1, 0.5 * h);
            momentum_step(&c, U1, Q1, (1.0 - 2.0 * lam) * h);
            link_step(&c.g, U1, Q1, 0.5 * h);
            momentum_step(&c, U1, Q1, lam * h);
        }
    }

    if (fermions) sf1 = fermion_solve(&c, U1);
    double k1 = ora_kinetic(dims, Q1), sg1 = ora_plaquette_action(dims, U1, beta);
    energies[0] = k0;
    energies[1] = sg0;
    energies[2] = sf0;
    energies[3] = k1;
    energies[4] = sg1;
    energies[5] = sf1;
    double dh = (k1 + sg1 + sf1) - (k0 + sg0 + sf0);
    *accepted = u < exp(-dh) ? 1 : 0;
    *cg_iters = c.iters;
    *cg_solves = c.solves;
    free(phi);
    free(c.chi);
    return c.fail ? 1 : 0;
}
