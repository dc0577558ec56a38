// multishift.hip -- several masses on one Krylov space (multi-shift CG).
//
// For M_i = m_i^2 - D_eo D_oe all systems share D_eo D_oe; they differ by a
// shift sigma_i = m_i^2 - m_0^2 >= 0 of the smallest mass m_0 (the base).
// CG on the base generates residuals r_k; the residual of shifted system i
// after k steps is zeta_k^i r_k (the Krylov space does not depend on the
// shift).  Writing the CG recurrences as a three-term recurrence for r_k and
// matching it with the shifted one gives, with alpha_k, beta_k of the base,
//   zeta_{k+1} = zeta_k zeta_{k-1} alpha_{k-1} /
//                [zeta_{k-1} alpha_{k-1} (1 + alpha_k sigma) + alpha_k beta_{k-1} (zeta_{k-1} - zeta_k)]
//   alpha^i_k = alpha_k zeta_{k+1} / zeta_k,  beta^i_k = beta_k (zeta_{k+1} / zeta_k)^2
//   x^i += alpha^i_k p^i,  p^i = zeta_{k+1} r_{k+1} + beta^i_k p^i
// (zeta_0 = zeta_{-1} = 1, alpha_{-1} = 1, beta_{-1} = 0).  A shifted system
// stops updating once |zeta| |r| meets the target.  This is the multi-mass
// solve a rational-approximation HMC needs for staggered fermions.
//
// One iteration: the base hop and fused normal operator (shared with the
// plain solver), a finalize for alpha and every zeta, the base update
// (x_0, r, |r|^2), a finalize for beta, and one kernel that advances every
// shifted solution x_i += alpha_i p_i with the p_i it reads anyway and then
// every search direction (one read of each p_i per iteration, not two).  The recurrence runs in FP64, or with the search
// directions and the operator in FP32 or FP16 storage and the residual and
// the solutions in FP32.  In the mixed recurrence the base system takes the
// reliable updates of the mixed-precision CG: every K iterations, or when
// |r| fell below delta max |r|, every solution is added into the caller's
// FP64 field (its FP32 part restarts from zero), the base residual is
// replaced by b - M_0 x_0 computed in FP64, and beta and every beta_i are
// recomputed from it (the shifted residuals stay zeta_i r, which the
// replacement keeps to the accuracy of the FP64 residual).  Afterwards every
// mass gets an FP64 true-residual check that also refines it with a
// warm-started CG (mixed precision with FP16 storage when the recurrence was
// mixed) if the recurrence left it above tol.
#include <algorithm>
#include <chrono>
#include <cmath>

#include "hop.hpp"

namespace lqs {

void launch_normal_dot_shape(const Gauge &gauge, const CgVectors &v, LaunchShape sh, hipStream_t s);
void cg_residual_group(Ctx &ctx, const Gauge &gauge, const CgVectors &v, int gate_mode, int mode, hipStream_t s);

static constexpr int MS_MAX = 16;
static constexpr int MS_BLOCK = 256;

struct ShiftState {
    double sigma;                    // m_i^2 - m_0^2
    double zeta, zeta_prev, zeta_next;
    double alpha, beta;
    int32_t active;                  // still above the target
    int32_t iters;
    int32_t xupd;                    // alpha was formed this iteration: x_i += alpha p_i is due
};

struct ShiftPtrs {
    char *x[MS_MAX + 1];             // solution of each shifted system (storage PR)
    char *p[MS_MAX + 1];             // search direction of each shifted system (storage PI)
    double *x64[MS_MAX + 1];         // mixed recurrence: the caller's FP64 solution it is added into
                                     // (entry nshift: the base, for the final flush)
};

__global__ void __launch_bounds__(1024) ms_finalize_dot(CgState *base, ShiftState *sh, int nshift,
                                                        const double *partials, int nblocks)
{
    CgState &S = *base;
    if (S.phase != CG_RUNNING) return;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nblocks; i += blockDim.x) acc += partials[i];
    const double pq = block_sum(acc);
    if (threadIdx.x != 0) return;
    for (int i = 0; i < nshift; ++i) sh[i].xupd = 0;
    if (!isfinite(pq)) {
        S.phase = CG_NONFINITE;
        return;
    }
    if (!(pq > 0.0)) {
        S.phase = CG_BREAKDOWN;
        return;
    }
    const double a_prev = S.alpha, b_prev = S.beta, a = S.rho / pq;
    for (int i = 0; i < nshift; ++i) {
        ShiftState &T = sh[i];
        if (!T.active) continue;
        const double z = T.zeta, zp = T.zeta_prev;
        const double den = zp * a_prev * (1.0 + a * T.sigma) + a * b_prev * (zp - z);
        const double zn = z * zp * a_prev / den;
        T.zeta_next = zn;
        T.alpha = a * zn / z;
        T.xupd = 1;
    }
    S.alpha = a;
}

// x_0 += alpha p_0, r -= alpha q, |r|^2 of the base.  p_0 and q are stored
// as PI, r and x_0 as PR; the arithmetic is FP64.
template <int PI, int PR>
__global__ void __launch_bounds__(MS_BLOCK) ms_update(int vh, char *x0, char *r, const char *p0, const char *q,
                                                      const CgState *base, double *partials)
{
    typedef typename RealOf<PR>::type TR;
    if (base->phase != CG_RUNNING) return;
    const double a = base->alpha;
    double local = 0.0;
    for (int cb = blockIdx.x * blockDim.x + threadIdx.x; cb < vh; cb += gridDim.x * blockDim.x) {
        const V3<double> pv = vcast<double>(SpinorIO<PI>::load(p0, vh, cb));
        const V3<double> qv = vcast<double>(SpinorIO<PI>::load(q, vh, cb));
        V3<double> xv = vcast<double>(SpinorIO<PR>::load(x0, vh, cb));
        V3<double> rv = vcast<double>(SpinorIO<PR>::load(r, vh, cb));
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            xv.c[c].re += a * pv.c[c].re;
            xv.c[c].im += a * pv.c[c].im;
            rv.c[c].re -= a * qv.c[c].re;
            rv.c[c].im -= a * qv.c[c].im;
        }
        const V3<TR> rs = vcast<TR>(rv);
#pragma unroll
        for (int c = 0; c < 3; ++c)
            local += (double)rs.c[c].re * (double)rs.c[c].re + (double)rs.c[c].im * (double)rs.c[c].im;
        SpinorIO<PR>::store(x0, vh, cb, vcast<TR>(xv));
        SpinorIO<PR>::store(r, vh, cb, rs);
    }
    const double s = block_sum(local);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ void __launch_bounds__(1024) ms_finalize_update(CgState *base, ShiftState *sh, int nshift,
                                                           const double *partials, int nblocks)
{
    CgState &S = *base;
    if (S.phase != CG_RUNNING) return;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nblocks; i += blockDim.x) acc += partials[i];
    const double r2 = block_sum(acc);
    if (threadIdx.x != 0) return;
    S.rho_old = S.rho;
    S.rho = r2;
    S.beta = r2 / S.rho_old;
    S.iters += 1;
    int any = 0;
    for (int i = 0; i < nshift; ++i) {
        ShiftState &T = sh[i];
        if (!T.active) continue;
        const double ratio = T.zeta_next / T.zeta;
        T.beta = S.beta * ratio * ratio;
        T.zeta_prev = T.zeta;
        T.zeta = T.zeta_next;
        T.iters += 1;
        if (T.zeta * T.zeta * r2 <= S.stop2) T.active = 0;
        any |= T.active;
    }
    S.since_rel += 1;
    if (!isfinite(r2)) {
        S.phase = CG_NONFINITE;
        return;
    }
    if (r2 > S.max_rho) S.max_rho = r2;
    if ((r2 <= S.stop2 && !any) || S.iters >= S.max_iter) {
        S.phase = CG_INNER_DONE;
        // mixed: the FP64 residual of the base decides (and resumes when it is above the target)
        if (S.rel_interval > 0) S.reliable_pending = 1;
        return;
    }
    if (S.rel_interval > 0 && (S.since_rel >= S.rel_interval || r2 < S.delta2 * S.max_rho)) S.reliable_pending = 1;
}

// Mixed recurrence, reliable update: add every FP32 solution into its FP64
// field and restart it from zero (gated: the base's update is pending, or
// gated = 0 at the end of the recurrence).
template <int PR>
__global__ void __launch_bounds__(MS_BLOCK) ms_accumulate(int vh, const ShiftPtrs *ptr, int nshift, const CgState *base,
                                                          int gated)
{
    typedef typename RealOf<PR>::type TR;
    if (gated && !base->reliable_pending) return;
    for (int cb = blockIdx.x * blockDim.x + threadIdx.x; cb < vh; cb += gridDim.x * blockDim.x)
        for (int i = 0; i < nshift; ++i) {
            V3<double> xv = SpinorIO<F64>::load(ptr->x64[i], vh, cb);
            const V3<double> lv = vcast<double>(SpinorIO<PR>::load(ptr->x[i], vh, cb));
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                xv.c[c].re += lv.c[c].re;
                xv.c[c].im += lv.c[c].im;
            }
            SpinorIO<F64>::store(ptr->x64[i], vh, cb, xv);
            SpinorIO<PR>::store(ptr->x[i], vh, cb, vzero<TR>());
        }
}

// after a reliable update of the base: beta_i = beta (zeta_{k+1} / zeta_k)^2
// with the base's new beta (the same value ms_finalize_update set otherwise)
__global__ void ms_rebeta(const CgState *base, ShiftState *sh, int nshift)
{
    if (threadIdx.x != 0 || base->phase != CG_RUNNING) return;
    for (int i = 0; i < nshift; ++i) {
        ShiftState &T = sh[i];
        if (!T.active) continue;
        const double ratio = T.zeta / T.zeta_prev;
        T.beta = base->beta * ratio * ratio;
    }
}

// x_i += alpha_i p_i at site cb, p_i already loaded
template <int PI, int PR>
__device__ __forceinline__ void ms_shift_x(const ShiftPtrs *ptr, int i, int vh, int cb, double ai, const V3<double> &pi)
{
    typedef typename RealOf<PR>::type TR;
    V3<double> xi = vcast<double>(SpinorIO<PR>::load(ptr->x[i], vh, cb));
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        xi.c[c].re += ai * pi.c[c].re;
        xi.c[c].im += ai * pi.c[c].im;
    }
    SpinorIO<PR>::store(ptr->x[i], vh, cb, vcast<TR>(xi));
}

// x_i += alpha_i p_i where alpha_i was formed this iteration; p_0 = r + beta p_0;
// p_i = zeta_i r + beta_i p_i for active shifts.  (One block grid per system
// instead of the loop over the shifts measured slower: 0.41 vs 0.37 s for 8
// masses on 64^3 x 16 in FP64, as every system re-read the residual.)
template <int PI, int PR>
__global__ void __launch_bounds__(MS_BLOCK) ms_pupdate(int vh, const char *r, char *p0, const ShiftPtrs *ptr,
                                                       int nshift, const CgState *base, const ShiftState *sh)
{
    typedef typename RealOf<PI>::type TI;
    if (base->phase != CG_RUNNING) return;
    const double b = base->beta;
    for (int cb = blockIdx.x * blockDim.x + threadIdx.x; cb < vh; cb += gridDim.x * blockDim.x) {
        const V3<double> rv = vcast<double>(SpinorIO<PR>::load(r, vh, cb));
        V3<double> pv = vcast<double>(SpinorIO<PI>::load(p0, vh, cb));
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            pv.c[c].re = rv.c[c].re + b * pv.c[c].re;
            pv.c[c].im = rv.c[c].im + b * pv.c[c].im;
        }
        SpinorIO<PI>::store(p0, vh, cb, vcast<TI>(pv));
        for (int i = 0; i < nshift; ++i) {
            const bool xu = sh[i].xupd != 0, act = sh[i].active != 0;
            if (!xu && !act) continue;
            V3<double> pi = vcast<double>(SpinorIO<PI>::load(ptr->p[i], vh, cb));
            if (xu) ms_shift_x<PI, PR>(ptr, i, vh, cb, sh[i].alpha, pi);
            if (!act) continue;
            const double z = sh[i].zeta, bi = sh[i].beta;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                pi.c[c].re = z * rv.c[c].re + bi * pi.c[c].re;
                pi.c[c].im = z * rv.c[c].im + bi * pi.c[c].im;
            }
            SpinorIO<PI>::store(ptr->p[i], vh, cb, vcast<TI>(pi));
        }
    }
}

// After the recurrence: the x_i updates of the last iteration, whose p-update
// was skipped because that iteration ended the recurrence (alpha_i formed,
// base no longer running).  Nothing to do while the base still runs (the
// iteration cap of the host loop): its p-update has applied them.
template <int PI, int PR>
__global__ void __launch_bounds__(MS_BLOCK) ms_xflush(int vh, const ShiftPtrs *ptr, int nshift, const CgState *base,
                                                      const ShiftState *sh)
{
    if (base->phase == CG_RUNNING) return;
    for (int cb = blockIdx.x * blockDim.x + threadIdx.x; cb < vh; cb += gridDim.x * blockDim.x)
        for (int i = 0; i < nshift; ++i) {
            if (!sh[i].xupd) continue;
            const V3<double> pi = vcast<double>(SpinorIO<PI>::load(ptr->p[i], vh, cb));
            ms_shift_x<PI, PR>(ptr, i, vh, cb, sh[i].alpha, pi);
        }
}

// x_0 = x_i = 0, r = p_0 = p_i = b, |b|^2 (of b in FP64)
template <int PI, int PR>
__global__ void __launch_bounds__(MS_BLOCK) ms_init(int vh, const double *b, char *x0, char *r, char *p0,
                                                    const ShiftPtrs *ptr, int nshift, double *partials)
{
    typedef typename RealOf<PI>::type TI;
    typedef typename RealOf<PR>::type TR;
    double local = 0.0;
    for (int cb = blockIdx.x * blockDim.x + threadIdx.x; cb < vh; cb += gridDim.x * blockDim.x) {
        const V3<double> bv = SpinorIO<F64>::load(b, vh, cb);
#pragma unroll
        for (int c = 0; c < 3; ++c) local += bv.c[c].re * bv.c[c].re + bv.c[c].im * bv.c[c].im;
        SpinorIO<PR>::store(x0, vh, cb, vzero<TR>());
        SpinorIO<PR>::store(r, vh, cb, vcast<TR>(bv));
        SpinorIO<PI>::store(p0, vh, cb, vcast<TI>(bv));
        for (int i = 0; i < nshift; ++i) {
            SpinorIO<PR>::store(ptr->x[i], vh, cb, vzero<TR>());
            SpinorIO<PI>::store(ptr->p[i], vh, cb, vcast<TI>(bv));
        }
    }
    const double s = block_sum(local);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ void __launch_bounds__(1024) ms_finalize_init(CgState *base, const double *partials, int nblocks)
{
    double acc = 0.0;
    for (int i = threadIdx.x; i < nblocks; i += blockDim.x) acc += partials[i];
    const double b2 = block_sum(acc);
    if (threadIdx.x != 0) return;
    CgState &S = *base;
    S.b2 = b2;
    S.stop2 *= b2;
    S.rho = b2;
    S.max_rho = b2;
    S.true_r2 = b2;
    S.alpha = 1.0;  // alpha_{-1}
    S.beta = 0.0;   // beta_{-1}
    S.phase = (b2 == 0.0) ? CG_CONVERGED : (isfinite(b2) ? CG_RUNNING : CG_NONFINITE);
}

void multishift_solve(Ctx &ctx, const Gauge &gauge, int nmass, const double *masses, const double *b, double *const *x,
                      const lqs_cg_params &prm, lqs_cg_stats *stats, hipStream_t s)
{
    auto t0 = std::chrono::steady_clock::now();
    LQS_REQUIRE(nmass >= 1 && nmass <= MS_MAX + 1, LQS_EINVAL, "multi-shift takes 1..17 masses");
    LQS_REQUIRE(prm.inner_prec == F64 || prm.inner_prec == F32 || prm.inner_prec == F16, LQS_EINVAL,
                "inner_prec must be LQS_F64, LQS_F32 or LQS_F16");
    const Geom &g = gauge.g;
    const int vh = (int)gauge.vh;
    int base = 0;
    for (int i = 1; i < nmass; ++i)
        if (masses[i] < masses[base]) base = i;
    std::vector<int> shifts;
    for (int i = 0; i < nmass; ++i)
        if (i != base) shifts.push_back(i);
    const int nshift = (int)shifts.size();

    // precisions of the recurrence: search directions and operator PI, residual PR
    const int PI = prm.inner_prec, PR = PI == F64 ? F64 : F32;
    const int64_t fi = field_bytes(g, PI, 1), fr = field_bytes(g, PR, 1);
    CgVectors v{};
    v.prec = PI;
    v.acc_prec = PR;
    v.recon = prm.inner_recon == 12 ? 12 : 18;
    v.nrhs = 1;
    v.mass = masses[base];
    v.p = ctx.workspace("ms.p", fi);
    v.q = ctx.workspace("ms.q", fi);
    v.t = ctx.workspace("ms.t", fi);
    v.r = ctx.workspace("ms.r", fr);
    // the recurrence's solutions: the caller's FP64 fields, or FP32 workspaces
    std::vector<char *> xr(nmass);
    for (int i = 0; i < nmass; ++i)
        xr[i] = PR == F64 ? (char *)x[i] : (char *)ctx.workspace("ms.x" + std::to_string(i), fr);
    const bool mixed = PR != F64;
    v.x = mixed ? x[base] : (double *)xr[base];
    v.xlo = xr[base];
    v.b = (double *)b;
    v.t64 = mixed ? ctx.workspace("ms.t64", field_bytes(g, F64, 1)) : nullptr;
    v.max_blocks = cg_partials_needed(gauge, 1);
    v.partials = (double *)ctx.workspace("ms.partials", sizeof(double) * (size_t)v.max_blocks);
    v.state = (CgState *)ctx.workspace("ms.state", sizeof(CgState));
    ShiftPtrs hp{};
    std::vector<ShiftState> hsh(nshift);
    for (int k = 0; k < nshift; ++k) {
        hp.x[k] = xr[shifts[k]];
        hp.x64[k] = x[shifts[k]];
        hp.p[k] = (char *)ctx.workspace("ms.p" + std::to_string(k), fi);
        ShiftState &T = hsh[k];
        T = ShiftState{};
        T.sigma = masses[shifts[k]] * masses[shifts[k]] - masses[base] * masses[base];
        T.zeta = T.zeta_prev = 1.0;
        T.active = 1;
    }
    ShiftPtrs *dp = (ShiftPtrs *)ctx.workspace("ms.ptrs", sizeof(ShiftPtrs));
    ShiftState *dsh = (ShiftState *)ctx.workspace("ms.shifts", sizeof(ShiftState) * (nshift > 0 ? nshift : 1));
    CgState S{};
    S.m2 = masses[base] * masses[base];
    S.stop2 = prm.tol * prm.tol;
    S.max_iter = prm.max_iter;
    S.phase = CG_RUNNING;
    if (mixed) {
        S.rel_interval = prm.reliable_interval > 0 ? prm.reliable_interval : 100;
        const double delta = prm.reliable_delta > 0 ? prm.reliable_delta : default_reliable_delta(PI);
        S.delta2 = delta * delta;
    }
    // the base as one more entry of the accumulation list (its FP32 and FP64 solutions)
    ShiftPtrs hall = hp;
    hall.x[nshift] = xr[base];
    hall.x64[nshift] = x[base];
    ShiftPtrs *dall = (ShiftPtrs *)ctx.workspace("ms.ptrs_all", sizeof(ShiftPtrs));
    if (mixed) LQS_HIP(hipMemcpyAsync(dall, &hall, sizeof(ShiftPtrs), hipMemcpyHostToDevice, s));
    LQS_HIP(hipMemcpyAsync(dp, &hp, sizeof(ShiftPtrs), hipMemcpyHostToDevice, s));
    if (nshift) LQS_HIP(hipMemcpyAsync(dsh, hsh.data(), sizeof(ShiftState) * nshift, hipMemcpyHostToDevice, s));
    LQS_HIP(hipMemcpyAsync(v.state, &S, sizeof(CgState), hipMemcpyHostToDevice, s));

    if (mixed)
        for (int i = 0; i < nmass; ++i) LQS_HIP(hipMemsetAsync(x[i], 0, field_bytes(g, F64, 1), s));
    int blocks = (vh + MS_BLOCK - 1) / MS_BLOCK;
    if (blocks > 1024) blocks = 1024;
#define LQS_MS_PREC(STMT)                                                                                         \
    if (PI == F64) {                                                                                              \
        constexpr int P_I = F64, P_R = F64;                                                                       \
        STMT;                                                                                                     \
    } else if (PI == F32) {                                                                                       \
        constexpr int P_I = F32, P_R = F32;                                                                       \
        STMT;                                                                                                     \
    } else {                                                                                                      \
        constexpr int P_I = F16, P_R = F32;                                                                       \
        STMT;                                                                                                     \
    }
    LQS_MS_PREC(hipLaunchKernelGGL((ms_init<P_I, P_R>), dim3(blocks), dim3(MS_BLOCK), 0, s, vh, b, xr[base], (char *)v.r,
                                   (char *)v.p, (const ShiftPtrs *)dp, nshift, v.partials));
    hipLaunchKernelGGL(ms_finalize_init, dim3(1), dim3(1024), 0, s, v.state, (const double *)v.partials, blocks);
    LQS_HIP(hipGetLastError());

    const LinkRef L = gauge.ref(PI, v.recon);
    const LaunchShape sh = default_hop_shape(L, 1);
    const int nd_blocks = (vh + sh.block - 1) / sh.block;
    CgState hs{};
    int64_t enqueued = 0;
    const int64_t cap = (int64_t)prm.max_iter + 64;
    while (true) {
        for (int i = 0; i < 8; ++i) {
            launch_hop_gated(g, L, PI, v.recon, 0, 1, 1, v.p, v.t, v.state, 1, sh, s);
            launch_normal_dot_shape(gauge, v, sh, s);
            hipLaunchKernelGGL(ms_finalize_dot, dim3(1), dim3(1024), 0, s, v.state, dsh, nshift,
                               (const double *)v.partials, nd_blocks);
            LQS_MS_PREC(hipLaunchKernelGGL((ms_update<P_I, P_R>), dim3(blocks), dim3(MS_BLOCK), 0, s, vh, xr[base],
                                           (char *)v.r, (const char *)v.p, (const char *)v.q,
                                           (const CgState *)v.state, v.partials));
            hipLaunchKernelGGL(ms_finalize_update, dim3(1), dim3(1024), 0, s, v.state, dsh, nshift,
                               (const double *)v.partials, blocks);
            if (mixed && (i & 3) == 3) {
                // reliable update (gated on the base's pending flag)
                hipLaunchKernelGGL((ms_accumulate<F32>), dim3(blocks), dim3(MS_BLOCK), 0, s, vh, (const ShiftPtrs *)dp,
                                   nshift, (const CgState *)v.state, 1);
                cg_residual_group(ctx, gauge, v, 2, 0, s);
                hipLaunchKernelGGL(ms_rebeta, dim3(1), dim3(64), 0, s, (const CgState *)v.state, dsh, nshift);
            }
            LQS_MS_PREC(hipLaunchKernelGGL((ms_pupdate<P_I, P_R>), dim3(blocks), dim3(MS_BLOCK), 0, s, vh,
                                           (const char *)v.r, (char *)v.p, (const ShiftPtrs *)dp, nshift,
                                           (const CgState *)v.state, (const ShiftState *)dsh));
            LQS_HIP(hipGetLastError());
        }
        enqueued += 8;
        LQS_HIP(hipMemcpyAsync(&hs, v.state, sizeof(CgState), hipMemcpyDeviceToHost, s));
        LQS_HIP(hipStreamSynchronize(s));
        if (hs.phase != CG_RUNNING || enqueued > cap) break;
    }
    if (nshift) {
        LQS_MS_PREC(hipLaunchKernelGGL((ms_xflush<P_I, P_R>), dim3(blocks), dim3(MS_BLOCK), 0, s, vh,
                                       (const ShiftPtrs *)dp, nshift, (const CgState *)v.state,
                                       (const ShiftState *)dsh));
    }
    LQS_HIP(hipGetLastError());
    if (nshift) LQS_HIP(hipMemcpyAsync(hsh.data(), dsh, sizeof(ShiftState) * nshift, hipMemcpyDeviceToHost, s));
    LQS_HIP(hipStreamSynchronize(s));

#undef LQS_MS_PREC
    if (mixed) {
        hipLaunchKernelGGL((ms_accumulate<F32>), dim3(blocks), dim3(MS_BLOCK), 0, s, vh, (const ShiftPtrs *)dall,
                           nshift + 1, (const CgState *)v.state, 0);
        LQS_HIP(hipGetLastError());
    }
    // every mass: FP64 true residual from its own solution, refined by a
    // warm-started CG (in the recurrence's precision, with reliable updates)
    // when the shared recurrence ended above the target.  The masses are
    // refined together as one block of CGs with one mass per column (up to 16
    // per block), so every hop reads the links once for all masses still
    // refining; a column that starts below the target does no iteration.
    lqs_cg_params rp = prm;
    rp.use_x0 = 1;
    rp.persistent = 0;
    // A refinement starts close to its solution (about 1e-7 relative after an
    // FP32 recurrence), where FP16 storage takes the same iterations as FP32 and
    // each is cheaper: after a mixed recurrence the refinement runs with FP16
    // storage when the gauge holds that format (measured, 64^3 x 16, 8 masses,
    // FP32 recurrence: 41 refinement iterations either way, 57 vs 71 ms).
    if (mixed && gauge.fmt[F16][v.recon == 12 ? 1 : 0]) rp.inner_prec = F16;
    const int64_t f64 = field_bytes(g, F64, 1);
    const int per_block = std::min(nmass, 16);
    char *xb = (char *)ctx.workspace("ms.xblock", f64 * per_block);
    char *bb = (char *)ctx.workspace("ms.bblock", f64 * per_block);
    for (int c0 = 0; c0 < nmass; c0 += per_block) {
        const int n = std::min(per_block, nmass - c0);
        for (int i = 0; i < n; ++i) {
            LQS_HIP(hipMemcpyAsync(xb + i * f64, x[c0 + i], f64, hipMemcpyDeviceToDevice, s));
            LQS_HIP(hipMemcpyAsync(bb + i * f64, b, f64, hipMemcpyDeviceToDevice, s));
        }
        lqs_problem pb{static_cast<const lqs_gauge *>(&gauge), masses[c0], n, (const double *)bb, (double *)xb};
        const std::vector<double> mcol(masses + c0, masses + c0 + n);
        cg_solve_one(ctx, pb, rp, stats + c0, s, &mcol);
        for (int i = 0; i < n; ++i)
            LQS_HIP(hipMemcpyAsync(x[c0 + i], xb + i * f64, f64, hipMemcpyDeviceToDevice, s));
    }
    LQS_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < nmass; ++i) {
        const int shared = (i == base) ? hs.iters : hsh[std::find(shifts.begin(), shifts.end(), i) - shifts.begin()].iters;
        stats[i].restarts += stats[i].iters > 0 ? 1 : 0;
        stats[i].iters += shared;
        if (hs.phase == CG_NONFINITE) stats[i].status = LQS_ENONFINITE;
    }
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int i = 0; i < nmass; ++i) {
        stats[i].seconds = secs;
        stats[i].device_seconds = 0.0;
        stats[i].gflops = stats[i].gbytes_per_s = 0.0;
    }
}

}  // namespace lqs
