/*
 * synth.c -- seeded synthetic inputs for the staggered even-odd solver.
 *
 * This module generates the gauge configurations and sources that both the
 * CPU oracle and the GPU library consume.  It holds none of the operator's
 * arithmetic: no Dirac operator, no phases, no solver.  Every value is a pure
 * function of (seed, site, direction, draw index), so the output does not
 * depend on the thread count or the loop order.
 *
 * Layouts (all complex numbers are (re, im) pairs of doubles, row-major 3x3):
 *   links   : [4][Nt][Nz][Ny][Nx][3][3]   direction mu = 0,1,2,3 is x,y,z,t
 *   sites   : [Nt][Nz][Ny][Nx][3][3]      one SU(3) matrix per site
 *   spinor  : [Nt][Nz][Ny][Nx][3]         one colour vector per site
 *
 * Random numbers: counter-based SplitMix64 (Steele, Lea, Flood, "Fast
 * splittable pseudorandom number generators", OOPSLA 2014).  Uniforms take the
 * top 53 bits; normals come from the Box-Muller transform.
 *
 * SU(3) generators:
 *   haar   : two rows of complex Gaussians, Gram-Schmidt orthonormalised, third
 *            row = conj(row1 x row2).  Right-invariant under SU(3), hence Haar.
 *   smooth : U = exp(i eps H), H = traceless Hermitian part of a 3x3 matrix of
 *            complex Gaussians; exp by scaling and squaring of a Taylor series,
 *            then the same row canonicalisation as haar so that rows 1-2
 *            determine row 3 exactly as a 12-real storage would rebuild it.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

typedef double complex cplx;

#define GOLDEN 0x9E3779B97F4A7C15ULL

static uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Draw number n of the stream identified by (seed, key). */
static uint64_t draw(uint64_t seed, uint64_t key, uint64_t n)
{
    uint64_t start = mix64(mix64(seed + GOLDEN) ^ (key * GOLDEN + 0x632BE59BD9B4E019ULL));
    return mix64(start + (n + 1) * GOLDEN);
}

/* Uniform in the open interval (0, 1). */
static double uniform(uint64_t seed, uint64_t key, uint64_t n)
{
    return ((double)(draw(seed, key, n) >> 11) + 0.5) * 0x1p-53;
}

/* Normals 2k and 2k+1 of the stream, one complex number with N(0,1) parts. */
static cplx cgauss(uint64_t seed, uint64_t key, uint64_t k)
{
    double u1 = uniform(seed, key, 2 * k);
    double u2 = uniform(seed, key, 2 * k + 1);
    double r = sqrt(-2.0 * log(u1));
    double th = 2.0 * M_PI * u2;
    return r * cos(th) + I * (r * sin(th));
}

/* Rows 0 and 1 orthonormalised in place, row 2 = conj(row0 x row1). */
static void canonicalise(cplx m[3][3])
{
    double n0 = 0.0;
    for (int j = 0; j < 3; ++j) n0 += creal(m[0][j] * conj(m[0][j]));
    n0 = 1.0 / sqrt(n0);
    for (int j = 0; j < 3; ++j) m[0][j] *= n0;
    cplx d = 0.0;
    for (int j = 0; j < 3; ++j) d += conj(m[0][j]) * m[1][j];
    for (int j = 0; j < 3; ++j) m[1][j] -= d * m[0][j];
    double n1 = 0.0;
    for (int j = 0; j < 3; ++j) n1 += creal(m[1][j] * conj(m[1][j]));
    n1 = 1.0 / sqrt(n1);
    for (int j = 0; j < 3; ++j) m[1][j] *= n1;
    m[2][0] = conj(m[0][1] * m[1][2] - m[0][2] * m[1][1]);
    m[2][1] = conj(m[0][2] * m[1][0] - m[0][0] * m[1][2]);
    m[2][2] = conj(m[0][0] * m[1][1] - m[0][1] * m[1][0]);
}

static void haar(uint64_t seed, uint64_t key, cplx m[3][3])
{
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j) m[i][j] = cgauss(seed, key, (uint64_t)(3 * i + j));
    canonicalise(m);
}

/* H = traceless Hermitian part of a matrix of complex Gaussians. */
static void algebra(uint64_t seed, uint64_t key, cplx h[3][3])
{
    cplx a[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) a[i][j] = cgauss(seed, key, (uint64_t)(3 * i + j));
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) h[i][j] = 0.5 * (a[i][j] + conj(a[j][i]));
    cplx tr = (h[0][0] + h[1][1] + h[2][2]) / 3.0;
    for (int i = 0; i < 3; ++i) h[i][i] -= tr;
}

static void matmul(cplx c[3][3], cplx a[3][3], cplx b[3][3])
{
    cplx t[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx s = 0.0;
            for (int k = 0; k < 3; ++k) s += a[i][k] * b[k][j];
            t[i][j] = s;
        }
    memcpy(c, t, sizeof(t));
}

/* exp(A) by scaling and squaring: A/2^s has norm <= 1/4, Taylor to 1e-17. */
static void expm3(cplx a[3][3], cplx e[3][3])
{
    double nrm = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) nrm += creal(a[i][j] * conj(a[i][j]));
    nrm = sqrt(nrm);
    int s = 0;
    while (nrm > 0.25) { nrm *= 0.5; ++s; }
    double scale = ldexp(1.0, -s);
    cplx b[3][3], term[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            b[i][j] = a[i][j] * scale;
            e[i][j] = (i == j) ? 1.0 : 0.0;
            term[i][j] = (i == j) ? 1.0 : 0.0;
        }
    for (int k = 1; k <= 18; ++k) {
        matmul(term, term, b);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                term[i][j] /= (double)k;
                e[i][j] += term[i][j];
            }
    }
    for (int q = 0; q < s; ++q) matmul(e, e, e);
}

static void smooth(uint64_t seed, uint64_t key, double eps, cplx m[3][3])
{
    cplx h[3][3], a[3][3];
    algebra(seed, key, h);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) a[i][j] = I * eps * h[i][j];
    expm3(a, m);
    canonicalise(m);
}

/*
 * Gauge field of 4*V links.  kind 0: identity, 1: Haar, 2: smooth(eps).
 * Link (mu, lex) draws from the stream keyed by mu*V + lex.
 */
void synth_gauge(const int32_t dims[4], int32_t kind, double eps, uint64_t seed, double *out)
{
    const long vol = (long)dims[0] * dims[1] * dims[2] * dims[3];
    cplx *u = (cplx *)out;
#pragma omp parallel for schedule(static)
    for (long l = 0; l < 4 * vol; ++l) {
        cplx m[3][3];
        if (kind == 1) {
            haar(seed, (uint64_t)l, m);
        } else if (kind == 2) {
            smooth(seed, (uint64_t)l, eps, m);
        } else {
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) m[i][j] = (i == j) ? 1.0 : 0.0;
        }
        memcpy(u + 9 * l, m, sizeof(m));
    }
}

/* One Haar SU(3) matrix per site (gauge transformations); stream key = lex. */
void synth_site_haar(const int32_t dims[4], uint64_t seed, double *out)
{
    const long vol = (long)dims[0] * dims[1] * dims[2] * dims[3];
    cplx *g = (cplx *)out;
#pragma omp parallel for schedule(static)
    for (long x = 0; x < vol; ++x) {
        cplx m[3][3];
        haar(seed, (uint64_t)x, m);
        memcpy(g + 9 * x, m, sizeof(m));
    }
}

/* The traceless Hermitian matrices behind synth_gauge(kind=2), for checks. */
void synth_gauge_algebra(const int32_t dims[4], uint64_t seed, double *out)
{
    const long vol = (long)dims[0] * dims[1] * dims[2] * dims[3];
    cplx *h = (cplx *)out;
#pragma omp parallel for schedule(static)
    for (long l = 0; l < 4 * vol; ++l) {
        cplx m[3][3];
        algebra(seed, (uint64_t)l, m);
        memcpy(h + 9 * l, m, sizeof(m));
    }
}

/*
 * Random su(3) momenta: Q = sum_a q_a T_a with T_a = i lambda_a / 2 (Gell-Mann
 * lambda_a) and eight independent N(0,1) coefficients q_a per link, i.e.
 * density ~ exp(tr Q^2).  Stream key = link index mu * V + lex.
 */
void synth_momenta(const int32_t dims[4], uint64_t seed, double *out)
{
    const long vol = (long)dims[0] * dims[1] * dims[2] * dims[3];
    cplx *q = (cplx *)out;
    const double r3 = 1.0 / sqrt(3.0);
#pragma omp parallel for schedule(static)
    for (long l = 0; l < 4 * vol; ++l) {
        double a[8];
        for (int k = 0; k < 4; ++k) {
            cplx g = cgauss(seed, (uint64_t)l, (uint64_t)k);
            a[2 * k] = creal(g);
            a[2 * k + 1] = cimag(g);
        }
        /* H = sum_a q_a lambda_a / 2 (Hermitian traceless), Q = i H */
        cplx h[9];
        h[0] = 0.5 * (a[2] + a[7] * r3);
        h[4] = 0.5 * (-a[2] + a[7] * r3);
        h[8] = -a[7] * r3;
        h[1] = 0.5 * (a[0] - I * a[1]);
        h[2] = 0.5 * (a[3] - I * a[4]);
        h[5] = 0.5 * (a[5] - I * a[6]);
        h[3] = conj(h[1]);
        h[6] = conj(h[2]);
        h[7] = conj(h[5]);
        for (int i = 0; i < 9; ++i) q[9 * l + i] = I * h[i];
    }
}

/*
 * Complex Gaussian colour vectors, N(0,1) real and imaginary parts.
 * parity 0 or 1 fills only sites with (x+y+z+t) of that parity and leaves the
 * others zero; parity -1 fills every site.  Stream key = lex.
 */
void synth_source(const int32_t dims[4], int32_t parity, uint64_t seed, double *out)
{
    const int nx = dims[0], ny = dims[1], nz = dims[2];
    const long vol = (long)dims[0] * dims[1] * dims[2] * dims[3];
    cplx *s = (cplx *)out;
#pragma omp parallel for schedule(static)
    for (long x = 0; x < vol; ++x) {
        long r = x;
        int c0 = (int)(r % nx); r /= nx;
        int c1 = (int)(r % ny); r /= ny;
        int c2 = (int)(r % nz); r /= nz;
        int c3 = (int)r;
        int par = (c0 + c1 + c2 + c3) & 1;
        for (int c = 0; c < 3; ++c)
            s[3 * x + c] = (parity < 0 || par == parity) ? cgauss(seed, (uint64_t)x, (uint64_t)c) : 0.0;
    }
}
