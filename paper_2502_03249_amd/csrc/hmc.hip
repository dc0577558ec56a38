// hmc.hip -- hybrid Monte Carlo around the staggered solver: the simulation
// layer that the paper's backends serve (Sec. 3: HMC, the gauge action and its
// derivatives; the inversion inside it is the dominant cost, Sec. 1).
//
// State in the canonical link layout [4][V][3][3] complex128 (the layout of
// lqs_gauge_create), momenta Q in the same layout (anti-Hermitian traceless).
//   S_g = beta sum_x sum_{mu<nu} (1 - Re tr P_{mu nu}(x) / 3)   (periodic links)
//   K   = -sum_links tr Q^2
//   S_f = phi^dag M^-1 phi,  phi = m eta_e - D_eo eta_o
//   dU/dtau = Q U,  dQ/dtau = -F/2,  F = F_g + F_f with
//   F_g = (beta/3) TA(U V) (V: staple sum), F_f = -TA(U Pi) (force.hip).
// One thread per site (action) or per link (force, update, kinetic energy);
// block partials are summed by one block in index order (deterministic).
#include <chrono>
#include <cmath>

#include "lqs_impl.hpp"

namespace lqs {

typedef Cx<double> Cd;
struct Mat {
    Cd e[3][3];
};

__device__ __forceinline__ Mat mat_load(const double2 *p)
{
    Mat m;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double2 d = p[3 * i + j];
            m.e[i][j] = {d.x, d.y};
        }
    return m;
}

__device__ __forceinline__ void mat_store(double2 *p, const Mat &m)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) p[3 * i + j] = make_double2(m.e[i][j].re, m.e[i][j].im);
}

// a b, a b^dag, a^dag b
template <bool DA, bool DB> __device__ __forceinline__ Mat mat_mul(const Mat &a, const Mat &b)
{
    Mat c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            Cd s = {0.0, 0.0};
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                Cd x = DA ? Cd{a.e[k][i].re, -a.e[k][i].im} : a.e[i][k];
                Cd y = DB ? Cd{b.e[j][k].re, -b.e[j][k].im} : b.e[k][j];
                s = cadd(s, cmul(x, y));
            }
            c.e[i][j] = s;
        }
    return c;
}

// Lexicographic index of x + step * mu-hat (periodic).
__device__ __forceinline__ int nbr(const Geom &g, int lex, int mu, int step)
{
    int c[4];
    int l = lex;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        c[i] = l % g.n[i];
        l /= g.n[i];
    }
    c[mu] += step;
    if (c[mu] < 0) c[mu] += g.n[mu];
    if (c[mu] >= g.n[mu]) c[mu] -= g.n[mu];
    return c[0] + g.n[0] * (c[1] + g.n[1] * (c[2] + g.n[2] * c[3]));
}

__device__ __forceinline__ const double2 *link_at(const double2 *U, int vol, int mu, int lex)
{
    return U + 9 * ((int64_t)mu * vol + lex);
}

constexpr int HMC_BLOCK = 256;
constexpr int HMC_MAX_PARTIALS = 4096;

// sum over sites of sum_{mu<nu} Re tr P_{mu nu}(x); one partial per block
__global__ void __launch_bounds__(HMC_BLOCK) plaquette_kernel(Geom g, int vol, const double2 *U, double *partials)
{
    double s = 0.0;
    for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < vol; x += gridDim.x * blockDim.x) {
#pragma unroll
        for (int mu = 0; mu < 3; ++mu) {
            const Mat um = mat_load(link_at(U, vol, mu, x));
            const int xm = nbr(g, x, mu, 1);
            for (int nu = mu + 1; nu < 4; ++nu) {
                const int xn = nbr(g, x, nu, 1);
                // P = U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
                const Mat a = mat_mul<false, false>(um, mat_load(link_at(U, vol, nu, xm)));
                const Mat b = mat_mul<false, false>(mat_load(link_at(U, vol, nu, x)), mat_load(link_at(U, vol, mu, xn)));
                // Re tr P = Re tr(a b^dag), b = U_nu(x) U_mu(x+nu)
                double t = 0.0;
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int k = 0; k < 3; ++k) t += a.e[i][k].re * b.e[i][k].re + a.e[i][k].im * b.e[i][k].im;
                s += t;
            }
        }
    }
    s = block_sum(s);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// -sum_links tr Q^2; one partial per block
__global__ void __launch_bounds__(HMC_BLOCK) kinetic_kernel(int64_t nlinks, const double2 *Q, double *partials)
{
    double s = 0.0;
    for (int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; l < nlinks; l += (int64_t)gridDim.x * blockDim.x) {
        const Mat q = mat_load(Q + 9 * l);
        // tr(Q Q) = sum_{ik} q_ik q_ki
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int k = 0; k < 3; ++k) s -= q.e[i][k].re * q.e[k][i].re - q.e[i][k].im * q.e[k][i].im;
    }
    s = block_sum(s);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// out[slot] = scale * (offset + sum of n partials), in index order
__global__ void __launch_bounds__(1024) hmc_finalize(const double *partials, int n, double offset, double scale,
                                                     double *out, int slot)
{
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += partials[i];
    s = block_sum(s);
    if (threadIdx.x == 0) out[slot] = scale * (offset + s);
}

// F_g = (beta/3) TA(U V) on link (x, mu); mode 0: out = coeff F_g, 1: out += coeff F_g.
// Three threads per link: thread slot k of a block handles the direction
// nu_k != mu (its upper and lower staple, four SU(3) products), the three
// staple sums meet in LDS, and the slot-0 wave forms U V and its traceless
// anti-Hermitian part.  A block covers 64 consecutive sites of one mu (one
// wave per slot), so every load of a wave is a contiguous run of links.
// PK: the links are read from the word-major FP64 18-real copy of the same
// links (block 2 mu + parity, word k of checkerboard site cb at k * pitch +
// cb), where a wave's load of one word is two contiguous 512-byte runs
// instead of 64 loads 144 bytes apart; the output stays canonical.
constexpr int GF_SITES = 64;

template <bool PK>
__device__ __forceinline__ Mat gf_link(const double2 *U, int vol, const double2 *P, int pitch, int mu, int parity,
                                       int lex)
{
    if constexpr (!PK) return mat_load(link_at(U, vol, mu, lex));
    const double2 *b = P + (int64_t)(2 * mu + parity) * 9 * pitch + (lex >> 1);
    Mat m;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const double2 d = b[(int64_t)k * pitch];
        m.e[k / 3][k % 3] = {d.x, d.y};
    }
    return m;
}

template <bool PK>
__global__ void __launch_bounds__(3 * GF_SITES) gauge_force_kernel(Geom g, int vol, const double2 *U, const double2 *P,
                                                                   int pitch, double beta, double coeff, int mode,
                                                                   double2 *out)
{
    __shared__ double2 part[3][9][GF_SITES];
    const int mu = blockIdx.y;
    const int slot = threadIdx.x / GF_SITES, lane = threadIdx.x % GF_SITES;
    const int x = blockIdx.x * GF_SITES + lane;
    const bool valid = x < vol;
    // parity of x; its one-step neighbours have the other parity, x + mu - nu the same
    int par = 0;
    if (PK && valid) {
        int l = x;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            par += l % g.n[i];
            l /= g.n[i];
        }
        par &= 1;
    }
    if (valid) {
        const int nu = slot + (slot >= mu ? 1 : 0);
        const int xm = nbr(g, x, mu, 1);
        // upper staple U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
        const int xn = nbr(g, x, nu, 1);
        Mat a = mat_mul<false, true>(gf_link<PK>(U, vol, P, pitch, nu, par ^ 1, xm),
                                     gf_link<PK>(U, vol, P, pitch, mu, par ^ 1, xn));
        a = mat_mul<false, true>(a, gf_link<PK>(U, vol, P, pitch, nu, par, x));
        // lower staple U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu)
        const int xd = nbr(g, x, nu, -1), xmd = nbr(g, xm, nu, -1);
        Mat b = mat_mul<true, true>(gf_link<PK>(U, vol, P, pitch, nu, par, xmd),
                                    gf_link<PK>(U, vol, P, pitch, mu, par ^ 1, xd));
        b = mat_mul<false, false>(b, gf_link<PK>(U, vol, P, pitch, nu, par ^ 1, xd));
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                part[slot][3 * i + j][lane] = make_double2(a.e[i][j].re + b.e[i][j].re, a.e[i][j].im + b.e[i][j].im);
    }
    __syncthreads();
    if (slot != 0 || !valid) return;
    double2 *o = out + 9 * ((int64_t)mu * vol + x);
    // accumulate mode: fetch the old record before the arithmetic (see force.hip)
    double2 prev[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) prev[k] = mode == 1 ? o[k] : make_double2(0.0, 0.0);
    Mat v;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double2 p0 = part[0][3 * i + j][lane], p1 = part[1][3 * i + j][lane], p2 = part[2][3 * i + j][lane];
            v.e[i][j] = {(p0.x + p1.x) + p2.x, (p0.y + p1.y) + p2.y};
        }
    const Mat w = mat_mul<false, false>(gf_link<PK>(U, vol, P, pitch, mu, par, x), v);
    // TA(W) = (W - W^dag)/2 - tr(W - W^dag)/6
    Mat t;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) t.e[i][j] = {0.5 * (w.e[i][j].re - w.e[j][i].re), 0.5 * (w.e[i][j].im + w.e[j][i].im)};
    const double tri = (t.e[0][0].im + t.e[1][1].im + t.e[2][2].im) / 3.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) t.e[i][i].im -= tri;
    const double c = coeff * beta / 3.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            o[3 * i + j] = make_double2(prev[3 * i + j].x + c * t.e[i][j].re, prev[3 * i + j].y + c * t.e[i][j].im);
}

// exp(A) for a 3x3 complex A: A is scaled by 2^-s so that its max-row-sum
// norm is at most 1/4, the Taylor polynomial of degree 16 is evaluated in
// Horner form (truncation below 1e-24), and the result squared s times.
__device__ __forceinline__ Mat mat_exp(const Mat &a0)
{
    double nrm = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        double r = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) r += sqrt(a0.e[i][j].re * a0.e[i][j].re + a0.e[i][j].im * a0.e[i][j].im);
        nrm = r > nrm ? r : nrm;
    }
    int s = 0;
    while (nrm > 0.25 && s < 60) {
        nrm *= 0.5;
        ++s;
    }
    const double sc = ldexp(1.0, -s);
    Mat a;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) a.e[i][j] = {a0.e[i][j].re * sc, a0.e[i][j].im * sc};
    // Horner: E = I + a/1 (I + a/2 (I + ... (I + a/16)))
    Mat e;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) e.e[i][j] = {i == j ? 1.0 : 0.0, 0.0};
    for (int k = 16; k >= 1; --k) {
        Mat t = mat_mul<false, false>(a, e);
        const double inv = 1.0 / k;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) e.e[i][j] = {(i == j ? 1.0 : 0.0) + t.e[i][j].re * inv, t.e[i][j].im * inv};
    }
    for (int k = 0; k < s; ++k) e = mat_mul<false, false>(e, e);
    return e;
}

// U = exp(eps Q) U on every link
__global__ void __launch_bounds__(HMC_BLOCK) link_update_kernel(int64_t nlinks, double2 *U, const double2 *Q, double eps)
{
    const int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (l >= nlinks) return;
    Mat q = mat_load(Q + 9 * l);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) q.e[i][j] = {eps * q.e[i][j].re, eps * q.e[i][j].im};
    const Mat e = mat_exp(q);
    mat_store(U + 9 * l, mat_mul<false, false>(e, mat_load(U + 9 * l)));
}

// phi = m eta_e - t (FP64 single-parity fields, double2[3][vh])
__global__ void __launch_bounds__(HMC_BLOCK) pseudofermion_kernel(int vh, double m, const double2 *eta_e,
                                                                  const double2 *t, double2 *phi)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 3 * vh) return;
    const double2 a = eta_e[i], b = t[i];
    phi[i] = make_double2(m * a.x - b.x, m * a.y - b.y);
}

// Start of the next solve from the last two solutions (linear extrapolation in
// molecular-dynamics time; successive solves are equally spaced, h/2 apart
// for Omelyan and h for leapfrog): c <- 2c - p, p <- c.
__global__ void __launch_bounds__(HMC_BLOCK) extrapolate_kernel(int64_t n, double2 *c, double2 *p)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double2 cv = c[i], pv = p[i];
    p[i] = cv;
    c[i] = make_double2(2.0 * cv.x - pv.x, 2.0 * cv.y - pv.y);
}

static int reduce_blocks(int64_t n)
{
    int64_t b = (n + HMC_BLOCK - 1) / HMC_BLOCK;
    return (int)(b > HMC_MAX_PARTIALS ? HMC_MAX_PARTIALS : (b < 1 ? 1 : b));
}

// out[slot] (device) = beta * sum_x sum_{mu<nu} (1 - Re tr P / 3)
void launch_gauge_action(Ctx &ctx, const Geom &g, const double *U, double beta, double *out, int slot, hipStream_t s)
{
    const int vol = 2 * g.vh;
    double *part = (double *)ctx.workspace("hmc.partials.a", sizeof(double) * HMC_MAX_PARTIALS);
    const int nb = reduce_blocks(vol);
    hipLaunchKernelGGL(plaquette_kernel, dim3(nb), dim3(HMC_BLOCK), 0, s, g, vol, (const double2 *)U, part);
    LQS_HIP(hipGetLastError());
    // beta * (6 V - sum / 3) = (-beta/3) * (-18 V + sum)
    hipLaunchKernelGGL(hmc_finalize, dim3(1), dim3(1024), 0, s, (const double *)part, nb, -18.0 * vol, -beta / 3.0,
                       out, slot);
    LQS_HIP(hipGetLastError());
}

void launch_kinetic(Ctx &ctx, const Geom &g, const double *Q, double *out, int slot, hipStream_t s)
{
    const int64_t nl = 4 * 2 * (int64_t)g.vh;
    double *part = (double *)ctx.workspace("hmc.partials.k", sizeof(double) * HMC_MAX_PARTIALS);
    const int nb = reduce_blocks(nl);
    hipLaunchKernelGGL(kinetic_kernel, dim3(nb), dim3(HMC_BLOCK), 0, s, nl, (const double2 *)Q, part);
    LQS_HIP(hipGetLastError());
    hipLaunchKernelGGL(hmc_finalize, dim3(1), dim3(1024), 0, s, (const double *)part, nb, 0.0, 1.0, out, slot);
    LQS_HIP(hipGetLastError());
}

void launch_gauge_force(const Geom &g, const double *U, double beta, double coeff, int accumulate, double *out,
                        hipStream_t s, const LinkRef *packed)
{
    const int vol = 2 * g.vh;
    dim3 grid((vol + GF_SITES - 1) / GF_SITES, 4);
    if (packed) {
        LQS_REQUIRE(!packed->temporal && packed->pitch >= g.vh && packed->block_bytes == 144 * (int64_t)packed->pitch,
                    LQS_EINVAL, "gauge force: packed links must be the plain FP64 18-real format");
        hipLaunchKernelGGL(gauge_force_kernel<true>, grid, dim3(3 * GF_SITES), 0, s, g, vol, (const double2 *)U,
                           (const double2 *)packed->base, (int)packed->pitch, beta, coeff, accumulate ? 1 : 0,
                           (double2 *)out);
    } else {
        hipLaunchKernelGGL(gauge_force_kernel<false>, grid, dim3(3 * GF_SITES), 0, s, g, vol, (const double2 *)U,
                           (const double2 *)nullptr, 0, beta, coeff, accumulate ? 1 : 0, (double2 *)out);
    }
    LQS_HIP(hipGetLastError());
}

void launch_link_update(const Geom &g, double *U, const double *Q, double eps, hipStream_t s)
{
    const int64_t nl = 4 * 2 * (int64_t)g.vh;
    hipLaunchKernelGGL(link_update_kernel, dim3((unsigned)((nl + HMC_BLOCK - 1) / HMC_BLOCK)), dim3(HMC_BLOCK), 0, s,
                       nl, (double2 *)U, (const double2 *)Q, eps);
    LQS_HIP(hipGetLastError());
}

// Repack every format the gauge holds from canonical links.
void gauge_repack(Gauge &gauge, const double *U, hipStream_t s)
{
    for (int prec = 0; prec < 3; ++prec)
        for (int rc = 0; rc < 2; ++rc)
            if (gauge.fmt[prec][rc])
                launch_pack_links(gauge.g, U, prec, rc ? 12 : 18, gauge.pitch, gauge.fmt[prec][rc], s);
}

// ---------------------------------------------------------------------------
// one trajectory

namespace {

// A gauge object over context workspaces (not freed by ~Gauge).
struct WsGauge {
    lqs_gauge g;
    WsGauge(Ctx &ctx, const Geom &geom, int inner_prec, int inner_recon)
    {
        g.ctx = &ctx;
        g.g = geom;
        g.vh = geom.vh;
        g.temporal = false;
        g.pitch = geom.vh;
        const int rcs[2] = {18, inner_recon};
        const int precs[2] = {F64, inner_prec};
        for (int k = 0; k < 2; ++k) {
            const int rc = rcs[k] == 12 ? 1 : 0;
            if (g.fmt[precs[k]][rc]) continue;
            const size_t bytes = (size_t)link_block_bytes_per_site(precs[k], rcs[k]) * g.pitch * 8;
            g.fmt[precs[k]][rc] = ctx.workspace(std::string("hmc.links.") + std::to_string(precs[k]) + "." +
                                                    std::to_string(rcs[k]),
                                                bytes);
        }
    }
    ~WsGauge()
    {
        for (auto &row : g.fmt)
            for (auto &p : row) p = nullptr;
    }
};

}  // namespace

void hmc_trajectory_impl(Ctx &ctx, const Geom &g, double *links, double *mom, const double *pf, double u,
                         const lqs_hmc_params &prm, lqs_hmc_stats &st, double *proposal, double *phi_out,
                         hipStream_t s)
{
    auto t0 = std::chrono::steady_clock::now();
    const int64_t vol = 2 * (int64_t)g.vh;
    const size_t link_bytes = sizeof(double) * 18 * 4 * (size_t)vol;
    const int64_t f64 = field_bytes(g, F64, 1);
    double *U1 = (double *)ctx.workspace("hmc.U1", link_bytes);
    double *scal = (double *)ctx.workspace("hmc.scalars", sizeof(double) * 16);
    LQS_HIP(hipMemcpyAsync(U1, links, link_bytes, hipMemcpyDeviceToDevice, s));
    const bool ferm = prm.fermions != 0;
    WsGauge wg(ctx, g, prm.cg.inner_prec, prm.cg.inner_recon);
    Gauge &gauge = wg.g;
    if (ferm) gauge_repack(gauge, U1, s);
    const LinkRef L64 = gauge.ref(F64, 18);
    const LaunchShape sh = default_hop_shape(L64, 1);

    double *phi = nullptr, *chi = nullptr, *psx = nullptr, *chi_prev = nullptr;
    int cg_solves = 0, cg_iters = 0, worst = LQS_OK;
    lqs_cg_params cgp = prm.cg;
    cgp.persistent = 0;
    const bool warm = prm.cg.use_x0 != 0;
    if (ferm) {
        phi = (double *)ctx.workspace("hmc.phi", f64);
        chi = (double *)ctx.workspace("hmc.chi", f64);
        chi_prev = (double *)ctx.workspace("hmc.chi_prev", f64);
        psx = (double *)ctx.workspace("hmc.psx", f64);
        LQS_HIP(hipMemsetAsync(chi, 0, f64, s));
        if (prm.fermions == 1) {
            double *eo = (double *)ctx.workspace("hmc.eta_o", f64);
            double *ee = (double *)ctx.workspace("hmc.eta_e", f64);
            launch_field_pack(g, pf, lqs_field{ee, F64, 0, 1}, s);
            launch_field_pack(g, pf, lqs_field{eo, F64, 1, 1}, s);
            // psx (even scratch) = D_eo eta_o
            launch_hop_gated(g, L64, F64, 18, 0, 0, 1, eo, psx, nullptr, 0, sh, s);
            hipLaunchKernelGGL(pseudofermion_kernel, dim3((3 * g.vh + HMC_BLOCK - 1) / HMC_BLOCK), dim3(HMC_BLOCK), 0,
                               s, (int)g.vh, prm.mass, (const double2 *)ee, (const double2 *)psx, (double2 *)phi);
            LQS_HIP(hipGetLastError());
        } else {
            launch_field_pack(g, pf, lqs_field{phi, F64, 0, 1}, s);
        }
        if (phi_out) {
            LQS_HIP(hipMemsetAsync(phi_out, 0, sizeof(double) * 6 * (size_t)vol, s));
            launch_field_unpack(g, lqs_field{phi, F64, 0, 1}, 1.0, phi_out, s);
        }
    }
    // chi = M^-1 phi on the current links (warm start from the previous chi if
    // asked); solves that only feed the force may use the looser force_tol
    int nsol = 0;
    auto solve = [&](bool energy) {
        lqs_problem pb{&wg.g, prm.mass, 1, phi, chi};
        lqs_cg_stats cs{};
        if (!warm) {
            LQS_HIP(hipMemsetAsync(chi, 0, f64, s));
        } else if (nsol == 1) {
            LQS_HIP(hipMemcpyAsync(chi_prev, chi, f64, hipMemcpyDeviceToDevice, s));
        } else if (nsol >= 2) {
            const int64_t n = 3 * (int64_t)g.vh;
            hipLaunchKernelGGL(extrapolate_kernel, dim3((unsigned)((n + HMC_BLOCK - 1) / HMC_BLOCK)), dim3(HMC_BLOCK), 0,
                               s, n, (double2 *)chi, (double2 *)chi_prev);
            LQS_HIP(hipGetLastError());
        }
        ++nsol;
        cgp.use_x0 = warm ? 1 : 0;
        cgp.tol = (energy || prm.force_tol <= 0) ? prm.cg.tol : prm.force_tol;
        cg_solve_one(ctx, pb, cgp, &cs, s);
        ++cg_solves;
        cg_iters += cs.iters;
        if (cs.status != LQS_OK && (worst == LQS_OK || cs.status < worst)) worst = cs.status;
    };
    // mom -= eps F / 2, the fermion part from chi on the current links; the
    // solve on the final links (last) also gives S_f at the end
    auto momentum = [&](double eps, bool have_chi, bool last) {
        // with fermions the word-major FP64 18-real copy of U1 is current here
        launch_gauge_force(g, U1, prm.beta, -0.5 * eps, 1, mom, s, ferm ? &L64 : nullptr);
        if (!ferm) return;
        if (!have_chi) solve(last);
        launch_hop_gated(g, L64, F64, 18, 0, 1, 1, chi, psx, nullptr, 0, sh, s);
        launch_force(g, L64, chi, chi, psx, psx, -0.5 * eps, 2, mom, s);
    };
    auto links_step = [&](double eps) {
        launch_link_update(g, U1, mom, eps, s);
        if (ferm) gauge_repack(gauge, U1, s);
    };

    // H at the start: scal[0..2] = K0, Sg0, Sf0
    launch_kinetic(ctx, g, mom, scal, 0, s);
    launch_gauge_action(ctx, g, U1, prm.beta, scal, 1, s);
    if (ferm) {
        solve(true);
        launch_field_dot(ctx, g, 1, phi, chi, scal + 8, s);
    }

    const double h = prm.tau / prm.nsteps;
    const double lam = prm.lambda > 0 ? prm.lambda : 0.1931833275037836;
    bool have_chi = ferm;  // chi belongs to the current links
    if (prm.integrator == LQS_LEAPFROG) {
        momentum(0.5 * h, have_chi, false);
        for (int k = 0; k < prm.nsteps; ++k) {
            links_step(h);
            const bool last = k == prm.nsteps - 1;
            momentum(last ? 0.5 * h : h, false, last);
        }
    } else {
        // consecutive lam*h updates at a step boundary act on the same links: merged
        double pending = lam * h;
        for (int k = 0; k < prm.nsteps; ++k) {
            momentum(pending, k == 0 && have_chi, false);
            links_step(0.5 * h);
            momentum((1.0 - 2.0 * lam) * h, false, false);
            links_step(0.5 * h);
            pending = 2.0 * lam * h;
        }
        momentum(lam * h, false, true);
    }
    // H at the end: chi is the solve on the final links (last momentum step)
    launch_kinetic(ctx, g, mom, scal, 3, s);
    launch_gauge_action(ctx, g, U1, prm.beta, scal, 4, s);
    if (ferm) launch_field_dot(ctx, g, 1, phi, chi, scal + 10, s);
    double hs[16];
    LQS_HIP(hipMemcpyAsync(hs, scal, sizeof(hs), hipMemcpyDeviceToHost, s));
    LQS_HIP(hipStreamSynchronize(s));
    st.k0 = hs[0];
    st.sg0 = hs[1];
    st.sf0 = ferm ? hs[8] : 0.0;
    st.k1 = hs[3];
    st.sg1 = hs[4];
    st.sf1 = ferm ? hs[10] : 0.0;
    st.dH = (st.k1 + st.sg1 + st.sf1) - (st.k0 + st.sg0 + st.sf0);
    st.accepted = (std::isfinite(st.dH) && u < std::exp(-st.dH)) ? 1 : 0;
    st.cg_solves = cg_solves;
    st.cg_iters = cg_iters;
    st.status = worst;
    if (proposal) LQS_HIP(hipMemcpyAsync(proposal, U1, link_bytes, hipMemcpyDeviceToDevice, s));
    if (st.accepted) LQS_HIP(hipMemcpyAsync(links, U1, link_bytes, hipMemcpyDeviceToDevice, s));
    // plaquette of the links returned: S_g = beta * 6V (1 - <P>) at beta = 1
    launch_gauge_action(ctx, g, links, 1.0, scal, 5, s);
    LQS_HIP(hipMemcpyAsync(hs, scal, sizeof(hs), hipMemcpyDeviceToHost, s));
    LQS_HIP(hipStreamSynchronize(s));
    st.plaquette = 1.0 - hs[5] / (6.0 * (double)vol);
    st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace lqs
