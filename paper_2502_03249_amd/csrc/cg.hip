// cg.hip -- conjugate gradient on the even-odd normal operator
// M = m^2 - D_eo D_oe (the inversion of Sec. 4.2), in FP64 or with a
// low-precision inner iteration and FP64 residual updates.
//
// Per iteration four kernels run back to back on one stream:
//   1. t = D_oe p                                      (hop)
//   2. q = m^2 p - D_eo t and <p,q>                     (hop + fused dot)
//   3. r -= alpha q and |r|^2                           (fused update + norm)
//   4. x += alpha p, p = r + beta p                     (one read of the old p)
// The dot products are reduced in two fixed-order stages (wave shuffles and
// LDS inside a block, then the last block to finish sums the block partials)
// and alpha, beta stay on the device; the host only polls the state record.
// Every few iterations a gated FP64 group runs between kernels 3 and 4:
//   x += alpha p                                        (the step 4 owes)
//   x += x_lo, x_lo = 0                                 (mixed precision)
//   t64 = D_oe x, r_hi = b - (m^2 x - D_eo t64), |r_hi|^2, r = r_hi
// It does nothing unless the state asks for it: after the iterated residual
// met the target (then it decides convergence on the FP64 residual), at the
// iteration cap, or in mixed precision every K iterations or when |r| fell
// below delta * max|r| (the reliable update of the mixed-precision solvers the
// paper cites, Clark et al. 2010).
#include <chrono>
#include <cmath>
#include <mutex>

#include "hop.hpp"

namespace lqs {

static constexpr int BLAS_BLOCK = 256;
static constexpr int MIN_HOP_BLOCK = 64;
// largest number of <p,q> partials the update kernel sums in every block
// (measured: folding pays on 32^4 and below, not on 64^3 x 16 with 8192)
static constexpr int FOLD_ALPHA_MAX = 2048;

// ---------------------------------------------------------------------------
// scalar bookkeeping, run by one thread of a one-block finalize kernel

__device__ void fin_alpha(CgState &S, double pq)
{
    if (!isfinite(pq)) S.phase = CG_NONFINITE;
    else if (!(pq > 0.0)) S.phase = CG_BREAKDOWN;
    else S.alpha = S.rho / pq;
}

__device__ void fin_update(CgState &S, double r2)
{
    S.rho_old = S.rho;
    S.rho = r2;
    S.beta = r2 / S.rho_old;
    S.iters += 1;
    S.since_rel += 1;
    if (!isfinite(r2)) {
        S.phase = CG_NONFINITE;
        return;
    }
    if (r2 > S.max_rho) S.max_rho = r2;
    if (r2 <= S.stop2 || S.iters >= S.max_iter) {
        S.phase = CG_INNER_DONE;
        S.reliable_pending = 1;
        return;
    }
    if (S.rel_interval > 0 && (S.since_rel >= S.rel_interval || r2 < S.delta2 * S.max_rho)) S.reliable_pending = 1;
}

// mode: 0 reliable update inside the iteration, 1 initial residual, 2 measure
// only, 3 periodic update with the reconstructed FP64 links (a residual that
// meets the target is handed on, still pending, to the mode-0 check with the
// stored links instead of ending the solve)
__device__ void fin_residual(CgState &S, double r2, int mode)
{
    S.true_r2 = r2;
    if (mode == 2) return;
    if (mode == 3 && isfinite(r2) && r2 <= S.stop2) {
        S.phase = CG_INNER_DONE;
        return;
    }
    if (mode == 1) {
        S.rho = r2;
        S.max_rho = r2;
        S.phase = isfinite(r2) ? (r2 <= S.stop2 ? CG_CONVERGED : CG_RUNNING) : CG_NONFINITE;
        return;
    }
    S.nreliable += 1;
    S.reliable_pending = 0;
    S.since_rel = 0;
    if (!isfinite(r2)) {
        S.phase = CG_NONFINITE;
    } else if (r2 <= S.stop2) {
        S.phase = CG_CONVERGED;
    } else if (S.iters >= S.max_iter) {
        S.phase = CG_MAXITER;
    } else if (S.rel_interval == 0) {
        // FP64 solver whose iterated residual drifted: restart from r = b - M x
        S.rho = r2;
        S.max_rho = r2;
        S.beta = 0.0;
        S.restarts += 1;
        S.phase = CG_RUNNING;
    } else {
        // mixed precision: continue with the FP64 residual, keep p
        S.beta = r2 / S.rho_old;
        S.rho = r2;
        S.max_rho = r2;
        S.phase = CG_RUNNING;
    }
}

// ---------------------------------------------------------------------------
// The new search direction r + beta p, in the accumulation precision (one
// fused multiply-add per component).

template <int PA>
__device__ __forceinline__ V3<typename RealOf<PA>::type> direction_of(const V3<typename RealOf<PA>::type> &rv,
                                                                      const V3<typename RealOf<PA>::type> &pv,
                                                                      typename RealOf<PA>::type beta)
{
    V3<typename RealOf<PA>::type> o;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        o.c[a].re = fused(beta, pv.c[a].re, rv.c[a].re);
        o.c[a].im = fused(beta, pv.c[a].im, rv.c[a].im);
    }
    return o;
}

// ---------------------------------------------------------------------------
// 2. q = m^2 p - D_eo t, <p, q>  (output parity even; t odd)

// FP16 storage: left alone the compiler gives the one-vector kernel 120 VGPRs
// (4 waves per SIMD); held to 6 waves it needs 62, without spills, and the
// 64^3x16 launch drops from 89.4 to 86.1 us (FP32/FP64 unchanged or slower).
// Not with LF_PREFETCH, whose words in flight need about 110 VGPRs.
template <int P, int R, int K, int LF>
__global__ void __launch_bounds__(512)
__attribute__((amdgpu_waves_per_eu((P == F16 && (LF & LF_PREFETCH) == 0) ? 6 : 1)))
normal_dot_kernel(Geom g, LinkRef L, const char *t, const char *p, char *q,
                                                         int64_t stride, CgState *st, double *partials,
                                                         int max_blocks, int nrhs, int ngroups, TileMap tmap)
{
    typedef typename RealOf<P>::type T;
    int grp;
    const int tile = tile_group(ngroups, tmap, g.n[3], grp);
    if (tile < 0 || tile * (int)blockDim.x >= g.vh) return;  // padding tile (whole block)
    const int cb = tile * blockDim.x + threadIdx.x;
    const bool valid = cb < g.vh;
    const int r0 = grp * K;
    bool blk[K], act[K];
    bool any = false;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        blk[j] = (r0 + j < nrhs) && st[r0 + j].phase == CG_RUNNING;
        act[j] = blk[j] && valid;
        any |= blk[j];
    }
    if (!any) return;  // uniform over the block
    extern __shared__ __align__(16) char win[];
    int w0 = 0, wlen = 0;
    const int wstride = lds_window_stride(g, P);
    if (LF & LF_LDS)
        stage_block_window<P, K>(g, tile * blockDim.x, t + r0 * stride, stride, blk, win, wstride, w0, wlen);
    double dot[K];
    V3<T> acc[K];
    // LF_PREFETCH with one vector: the site's own p is requested with the hop's words
    constexpr bool PF1 = (LF & LF_PREFETCH) != 0 && K == 1;
    typename SpinorIO<P>::Raw praw{};
    if (PF1 && act[0]) praw = SpinorIO<P>::load_raw(p + r0 * stride, g.vh, cb);
    if (valid) {
        const Site s = decode(g, cb, 0);
        hop_site<P, R, K, LF>(g, L, 0, s, cb, t + r0 * stride, stride, act, acc, win, wstride, w0, wlen);
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
        dot[j] = 0.0;
        if (!act[j]) continue;
        const V3<T> pv = PF1 ? SpinorIO<P>::decode(praw) : SpinorIO<P>::load(p + (r0 + j) * stride, g.vh, cb);
        const T m2 = (T)st[r0 + j].m2;
        V3<T> qv;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            qv.c[a].re = m2 * pv.c[a].re - acc[j].c[a].re;
            qv.c[a].im = m2 * pv.c[a].im - acc[j].c[a].im;
            dot[j] += (double)pv.c[a].re * (double)qv.c[a].re + (double)pv.c[a].im * (double)qv.c[a].im;
        }
        SpinorIO<P>::store(q + (r0 + j) * stride, g.vh, cb, qv);
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (!blk[j]) continue;
        const int r = r0 + j;
        const double s = block_sum(dot[j]);
        if (threadIdx.x == 0) partials[(int64_t)r * max_blocks + tile] = s;
    }
}

// ---------------------------------------------------------------------------
// 3. alpha = rho / <p, q>; r -= alpha q, |r|^2
//    (grid-stride, blockIdx.y = rhs; x += alpha p is left to the p-update,
//    which reads p anyway, or to the FP64 group's flush when that runs first)
//
// With nd_blocks > 0 every block sums the normal kernel's <p, q> partials
// itself, in the same order, so all blocks hold the same alpha without a
// separate reduction kernel (used while the partials are few; beyond
// FOLD_ALPHA_MAX of them the redundant sums cost more than the finalize
// kernel they replace, and FIN_DOT sets alpha instead).  Within this kernel
// no block reads a state field that another block writes: rho and phase are
// read, block 0 writes alpha and, on a breakdown (which every block detects
// by itself), the phase.  A thread requests the operands of its first site
// before the gate and the alpha reduction, whose memory round trips then
// overlap with them (on small lattices that is its only site).

template <int PA, int PI>
__global__ void __launch_bounds__(BLAS_BLOCK) update_kernel(int vh, char *r, const char *q, int64_t sa, int64_t si,
                                                            CgState *st, const double *pq_partials, int nd_blocks,
                                                            double *partials, int max_blocks)
{
    typedef typename RealOf<PA>::type T;
    const int rhs = blockIdx.y;
    CgState &S = st[rhs];
    r += rhs * sa;
    q += rhs * si;
    const int stride = gridDim.x * blockDim.x;
    const int c0 = blockIdx.x * blockDim.x + threadIdx.x;
    const int cf = c0 < vh ? c0 : vh - 1;  // a valid site for every thread (vh >= 1)
    const typename SpinorIO<PI>::Raw qraw = SpinorIO<PI>::load_raw(q, vh, cf);
    const typename SpinorIO<PA>::Raw rraw = SpinorIO<PA>::load_raw(r, vh, cf);
    const int phase = S.phase;
    issue_here(qraw);
    issue_here(rraw);
    if (phase != CG_RUNNING) return;
    double alpha_d = S.alpha;  // nd_blocks == 0: set by the FIN_DOT finalize
    if (nd_blocks > 0) {
        double acc = 0.0;
        for (int i = threadIdx.x; i < nd_blocks; i += blockDim.x) acc += pq_partials[(int64_t)rhs * max_blocks + i];
        const double pq = block_sum(acc);
        const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
        if (!isfinite(pq) || !(pq > 0.0)) {
            if (lead) S.phase = isfinite(pq) ? CG_BREAKDOWN : CG_NONFINITE;
            return;
        }
        alpha_d = S.rho / pq;
        if (lead) S.alpha = alpha_d;
    }
    const T alpha = (T)alpha_d;
    double local = 0.0;
    auto site = [&](int cb, const V3<T> &qv, V3<T> rv) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            rv.c[a].re = fused(-alpha, qv.c[a].re, rv.c[a].re);
            rv.c[a].im = fused(-alpha, qv.c[a].im, rv.c[a].im);
            local += (double)rv.c[a].re * (double)rv.c[a].re + (double)rv.c[a].im * (double)rv.c[a].im;
        }
        SpinorIO<PA>::store(r, vh, cb, rv);
    };
    if (c0 < vh) site(c0, vcast<T>(SpinorIO<PI>::decode(qraw)), SpinorIO<PA>::decode(rraw));
    for (int cb = c0 + stride; cb < vh; cb += stride)
        site(cb, vcast<T>(SpinorIO<PI>::load(q, vh, cb)), SpinorIO<PA>::load(r, vh, cb));
    const double s = block_sum(local);
    if (threadIdx.x == 0) partials[(int64_t)rhs * max_blocks + blockIdx.x] = s;
}

// ---------------------------------------------------------------------------
// 4. x += alpha p (x_lo in mixed precision), p = r + beta p
//
// The x update belongs to this iteration's alpha and the p before this
// kernel; it is skipped when the FP64 group ran after the update kernel
// (since_rel == 0: its flush already applied it).  No block writes the state.
// (As in the update kernel, the first site's operands are requested before
// the gate.)
template <int PA, int PI>
__device__ __forceinline__ void x_step(V3<typename RealOf<PA>::type> &xv, const V3<typename RealOf<PA>::type> &pv,
                                       typename RealOf<PA>::type alpha)
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        xv.c[a].re = fused(alpha, pv.c[a].re, xv.c[a].re);
        xv.c[a].im = fused(alpha, pv.c[a].im, xv.c[a].im);
    }
}

template <int PA, int PI>
__global__ void __launch_bounds__(BLAS_BLOCK) pupdate_kernel(int vh, char *x, const char *r, char *p, int64_t sa,
                                                             int64_t si, const CgState *st)
{
    typedef typename RealOf<PA>::type T;
    typedef typename RealOf<PI>::type TI;
    const int rhs = blockIdx.y;
    const CgState &S = st[rhs];
    x += rhs * sa;
    r += rhs * sa;
    p += rhs * si;
    const int stride = gridDim.x * blockDim.x;
    const int c0 = blockIdx.x * blockDim.x + threadIdx.x;
    const int cf = c0 < vh ? c0 : vh - 1;
    const typename SpinorIO<PA>::Raw rraw = SpinorIO<PA>::load_raw(r, vh, cf);
    const typename SpinorIO<PI>::Raw praw = SpinorIO<PI>::load_raw(p, vh, cf);
    const typename SpinorIO<PA>::Raw xraw = SpinorIO<PA>::load_raw(x, vh, cf);
    const int phase = S.phase;
    const bool xstep = S.since_rel != 0;
    const T beta = (T)S.beta, alpha = (T)S.alpha;
    issue_here(rraw);
    issue_here(praw);
    issue_here(xraw);
    if (phase != CG_RUNNING) return;
    auto site = [&](int cb, const V3<T> &rv, const V3<T> &pv, V3<T> xv) {
        if (xstep) {
            x_step<PA, PI>(xv, pv, alpha);
            SpinorIO<PA>::store(x, vh, cb, xv);
        }
        SpinorIO<PI>::store(p, vh, cb, vcast<TI>(direction_of<PA>(rv, pv, beta)));
    };
    if (c0 < vh)
        site(c0, SpinorIO<PA>::decode(rraw), vcast<T>(SpinorIO<PI>::decode(praw)), SpinorIO<PA>::decode(xraw));
    for (int cb = c0 + stride; cb < vh; cb += stride)
        site(cb, SpinorIO<PA>::load(r, vh, cb), vcast<T>(SpinorIO<PI>::load(p, vh, cb)),
             xstep ? SpinorIO<PA>::load(x, vh, cb) : vzero<T>());
}

// FP64 group, first: x += alpha p for the iteration whose p-update has not
// run yet (gate: reliable pending), with the p-update's arithmetic.
template <int PA, int PI>
__global__ void __launch_bounds__(BLAS_BLOCK) xflush_kernel(int vh, char *x, const char *p, int64_t sa, int64_t si,
                                                            const CgState *st)
{
    typedef typename RealOf<PA>::type T;
    const int rhs = blockIdx.y;
    const CgState &S = st[rhs];
    if (!S.reliable_pending) return;
    const T alpha = (T)S.alpha;
    x += rhs * sa;
    p += rhs * si;
    for (int cb = blockIdx.x * blockDim.x + threadIdx.x; cb < vh; cb += gridDim.x * blockDim.x) {
        V3<T> xv = SpinorIO<PA>::load(x, vh, cb);
        x_step<PA, PI>(xv, vcast<T>(SpinorIO<PI>::load(p, vh, cb)), alpha);
        SpinorIO<PA>::store(x, vh, cb, xv);
    }
}

// ---------------------------------------------------------------------------
// FP64 group: x += x_lo, x_lo = 0   (gate: 1 = reliable pending, 0 = always)

template <int PA>
__global__ void __launch_bounds__(BLAS_BLOCK) accumulate_kernel(int vh, double *x, char *xlo, int64_t sa,
                                                                const CgState *st, int gated)
{
    const int rhs = blockIdx.y;
    if (gated && !st[rhs].reliable_pending) return;
    char *xd = (char *)x + rhs * spinor_bytes_per_site(F64) * (int64_t)vh;
    xlo += rhs * sa;
    for (int cb = blockIdx.x * blockDim.x + threadIdx.x; cb < vh; cb += gridDim.x * blockDim.x) {
        V3<double> xv = SpinorIO<F64>::load(xd, vh, cb);
        const V3<double> lv = vcast<double>(SpinorIO<PA>::load(xlo, vh, cb));
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            xv.c[a].re += lv.c[a].re;
            xv.c[a].im += lv.c[a].im;
        }
        SpinorIO<F64>::store(xd, vh, cb, xv);
        SpinorIO<PA>::store(xlo, vh, cb, vcast<typename RealOf<PA>::type>(vzero<double>()));
    }
}

// r_hi = b - (m^2 x - D_eo t64) in FP64, |r_hi|^2; r (PA) = r_hi unless mode 2.
// gate_mode as in gate_state (0: all right-hand sides).
template <int R, int PA, int K, int LF>
__global__ void __launch_bounds__(512) residual_kernel(Geom g, LinkRef L, const char *t64, const char *x,
                                                       const char *b, char *r, int64_t sa, CgState *st,
                                                       double *partials, int max_blocks, int nrhs, int gate_mode,
                                                       int mode)
{
    const int64_t s64 = spinor_bytes_per_site(F64) * (int64_t)g.vh;
    const int cb = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = cb < g.vh;
    const int r0 = blockIdx.y * K;
    bool blk[K], act[K];
    bool any = false;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        blk[j] = (r0 + j < nrhs) && gate_state(st[r0 + j], gate_mode);
        act[j] = blk[j] && valid;
        any |= blk[j];
    }
    if (!any) return;
    V3<double> acc[K];
    double nrm[K];
    if (valid) {
        const Site s = decode(g, cb, 0);
        hop_site<F64, R, K, LF>(g, L, 0, s, cb, t64 + r0 * s64, s64, act, acc);
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
        nrm[j] = 0.0;
        if (!act[j]) continue;
        const V3<double> xv = SpinorIO<F64>::load(x + (r0 + j) * s64, g.vh, cb);
        const V3<double> bv = SpinorIO<F64>::load(b + (r0 + j) * s64, g.vh, cb);
        const double m2 = st[r0 + j].m2;
        V3<double> rv;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            rv.c[a].re = bv.c[a].re - (m2 * xv.c[a].re - acc[j].c[a].re);
            rv.c[a].im = bv.c[a].im - (m2 * xv.c[a].im - acc[j].c[a].im);
            nrm[j] += rv.c[a].re * rv.c[a].re + rv.c[a].im * rv.c[a].im;
        }
        if (mode != 2) SpinorIO<PA>::store(r + (r0 + j) * sa, g.vh, cb, vcast<typename RealOf<PA>::type>(rv));
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (!blk[j]) continue;
        const int rr = r0 + j;
        const double s = block_sum(nrm[j]);
        if (threadIdx.x == 0) partials[(int64_t)rr * max_blocks + blockIdx.x] = s;
    }
}

// |b|^2 per right-hand side; cold start: x = 0, r = b, p = b, x_lo = 0.
template <int PA, int PI>
__global__ void __launch_bounds__(BLAS_BLOCK) init_kernel(int vh, const char *b, double *x, char *r, char *p,
                                                          char *xlo, int64_t sa, int64_t si, CgState *st,
                                                          double *partials, int max_blocks, int cold)
{
    typedef typename RealOf<PA>::type T;
    typedef typename RealOf<PI>::type TI;
    const int rhs = blockIdx.y;
    const int64_t s64 = spinor_bytes_per_site(F64) * (int64_t)vh;
    b += rhs * s64;
    char *xd = (char *)x + rhs * s64;
    double local = 0.0;
    for (int cb = blockIdx.x * blockDim.x + threadIdx.x; cb < vh; cb += gridDim.x * blockDim.x) {
        const V3<double> bv = SpinorIO<F64>::load(b, vh, cb);
#pragma unroll
        for (int a = 0; a < 3; ++a) local += bv.c[a].re * bv.c[a].re + bv.c[a].im * bv.c[a].im;
        if (cold) {
            SpinorIO<F64>::store(xd, vh, cb, vzero<double>());
            SpinorIO<PA>::store(r + rhs * sa, vh, cb, vcast<T>(bv));
            SpinorIO<PI>::store(p + rhs * si, vh, cb, vcast<TI>(bv));
        }
        if (xlo) SpinorIO<PA>::store(xlo + rhs * sa, vh, cb, vzero<T>());
    }
    const double s = block_sum(local);
    if (threadIdx.x == 0) partials[(int64_t)rhs * max_blocks + blockIdx.x] = s;
}

// ---------------------------------------------------------------------------
// Second reduction stage: one block per right-hand side sums the block
// partials of the kernel before it in a fixed order and updates the scalars.
// Running it as its own kernel (rather than in the last block of the
// producer) needs no device-scope fence: the kernel boundary orders the
// partials' stores before these loads.

enum FinMode { FIN_DOT = 0, FIN_UPDATE = 1, FIN_RESID = 2, FIN_INIT = 3 };

__global__ void __launch_bounds__(1024) finalize_kernel(CgState *st, const double *partials, int max_blocks,
                                                       int nblocks, int mode, int gate_mode, int sub)
{
    const int r = blockIdx.x;
    // The state record (into registers) and the partials are requested
    // together, before the gate decides: one memory round trip instead of
    // three (gate, partials, then the fields the bookkeeping reads).  The
    // record is written back whole by thread 0.
    const double *p = partials + (int64_t)r * max_blocks;
    const int i0 = threadIdx.x;
    const double first = p[i0 < nblocks ? i0 : nblocks - 1];  // nblocks >= 1
    CgState S = st[r];
    double acc = 0.0;
    acc += i0 < nblocks ? first : 0.0;
    for (int i = i0 + blockDim.x; i < nblocks; i += blockDim.x) acc += p[i];
    bool active = true;
    if (mode == FIN_DOT || mode == FIN_UPDATE) active = S.phase == CG_RUNNING;
    else if (mode == FIN_RESID) active = gate_state(S, gate_mode);
    if (!active) return;
    const double v = block_sum(acc);
    if (threadIdx.x != 0) return;
    if (mode == FIN_DOT) {
        fin_alpha(S, v);
    } else if (mode == FIN_UPDATE) {
        fin_update(S, v);
    } else if (mode == FIN_RESID) {
        fin_residual(S, v, sub);
    } else {  // FIN_INIT, sub = cold start
        S.b2 = v;
        S.stop2 = S.stop2 * v;  // the host stored tol^2 here
        if (sub) {
            S.rho = v;
            S.max_rho = v;
            S.true_r2 = v;
            S.phase = (v == 0.0) ? CG_CONVERGED : (isfinite(v) ? CG_RUNNING : CG_NONFINITE);
        }
    }
    st[r] = S;
}

static void launch_finalize(const CgVectors &v, const double *partials, int nblocks, int mode, int gate_mode, int sub,
                            hipStream_t s)
{
    hipLaunchKernelGGL(finalize_kernel, dim3(v.nrhs), dim3(1024), 0, s, v.state, partials, v.max_blocks, nblocks,
                       mode, gate_mode, sub);
    LQS_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// host side

static int blas_blocks(int64_t vh)
{
    int64_t b = (vh + BLAS_BLOCK - 1) / BLAS_BLOCK;
    return (int)(b < 1024 ? b : 1024);
}

void cg_fill_rates(lqs_cg_stats &o, const Gauge &gauge, int prec, int recon, int nrhs)
{
    const double t = o.device_seconds > 0 ? o.device_seconds : o.seconds;
    if (!(t > 0) || o.iters <= 0) {
        o.gflops = o.gbytes_per_s = 0.0;
        return;
    }
    const double real = prec == F64 ? 8 : prec == F32 ? 4 : 2;
    const double lps = gauge.temporal ? 6.0 + 2.0 / gauge.g.n[3] : 8.0;
    const double L = lps * real * recon / (nrhs > 0 ? nrhs : 1);
    const double sv = (double)spinor_bytes_per_site(prec), a = (double)spinor_bytes_per_site(prec == F64 ? F64 : F32);
    // t = D_oe p; q = m^2 p - D_eo t; r updated from q; x and p updated from r and p
    const double bytes = (L + 2 * sv) + (L + 3 * sv) + (2 * a + sv) + (3 * a + 2 * sv);
    const double n = (double)gauge.vh * o.iters;
    o.gflops = 1140.0 * n / t * 1e-9;
    o.gbytes_per_s = bytes * n / t * 1e-9;
}

int cg_partials_needed(const Gauge &gauge, int nrhs)
{
    (void)nrhs;
    int64_t hop_blocks = (gauge.vh + MIN_HOP_BLOCK - 1) / MIN_HOP_BLOCK;
    return (int)(hop_blocks > 1024 ? hop_blocks : 1024);
}

template <int P, int R>
static void launch_normal_dot(const Gauge &gauge, const CgVectors &v, LaunchShape sh, hipStream_t s)
{
    const Geom &g = gauge.g;
    const int64_t stride = field_bytes(g, P, 1);
    const LinkRef L = gauge.ref(P, R);
    const int G = (v.nrhs + sh.rhs_per_thread - 1) / sh.rhs_per_thread;
    const TileMap tmap = tile_map(g, sh.block, sh.xcd_slab, time_run(g, sh.block, v.nrhs, P, sh.trun));
    const dim3 grid(tile_map_blocks(g, sh.block, tmap, G));
    const size_t lds = hop_lds_bytes(g, P, sh.rhs_per_thread, sh);
#define LQS_ND(K, LF)                                                                                             \
    hipLaunchKernelGGL((normal_dot_kernel<P, R, K, LF>), grid, dim3(sh.block), lds, s, g, L, (const char *)v.t,   \
                       (const char *)v.p, (char *)v.q, stride, v.state, v.partials,          \
                       v.max_blocks, v.nrhs, G, tmap)
#define LQS_ND_LF(LF)                                                                                            \
    if (sh.rhs_per_thread == 1) LQS_ND(1, LF);                                                                   \
    else if (sh.rhs_per_thread == 2) LQS_ND(2, LF);                                                              \
    else LQS_ND(4, LF)
    const int lf = (L.temporal ? LF_TEMPORAL : 0) | (sh.stream_links ? LF_STREAM : 0) | (lds ? LF_LDS : 0);
    if (sh.prefetch && !lds) {
        switch (lf) {
        case 0: LQS_ND_LF(LF_PREFETCH); break;
        case LF_TEMPORAL: LQS_ND_LF(LF_PREFETCH | LF_TEMPORAL); break;
        case LF_STREAM: LQS_ND_LF(LF_PREFETCH | LF_STREAM); break;
        default: LQS_ND_LF(LF_PREFETCH | LF_TEMPORAL | LF_STREAM); break;
        }
        LQS_HIP(hipGetLastError());
        return;
    }
    switch (lf) {
    case 0: LQS_ND_LF(0); break;
    case LF_TEMPORAL: LQS_ND_LF(LF_TEMPORAL); break;
    case LF_STREAM: LQS_ND_LF(LF_STREAM); break;
    case LF_TEMPORAL | LF_STREAM: LQS_ND_LF(LF_TEMPORAL | LF_STREAM); break;
    case LF_LDS: LQS_ND_LF(LF_LDS); break;
    case LF_LDS | LF_STREAM: LQS_ND_LF(LF_LDS | LF_STREAM); break;
    case LF_LDS | LF_TEMPORAL: LQS_ND_LF(LF_LDS | LF_TEMPORAL); break;
    default: LQS_ND_LF(LF_LDS | LF_TEMPORAL | LF_STREAM); break;
    }
#undef LQS_ND_LF
#undef LQS_ND
    LQS_HIP(hipGetLastError());
}

void launch_normal_dot_shape(const Gauge &gauge, const CgVectors &v, LaunchShape shd, hipStream_t s)
{
    if (v.prec == F64 && v.recon == 18) launch_normal_dot<F64, 18>(gauge, v, shd, s);
    else if (v.prec == F64) launch_normal_dot<F64, 12>(gauge, v, shd, s);
    else if (v.prec == F32 && v.recon == 18) launch_normal_dot<F32, 18>(gauge, v, shd, s);
    else if (v.prec == F32) launch_normal_dot<F32, 12>(gauge, v, shd, s);
    else if (v.recon == 18) launch_normal_dot<F16, 18>(gauge, v, shd, s);
    else launch_normal_dot<F16, 12>(gauge, v, shd, s);
}

// which 0: update (alpha from the nd_blocks <p,q> partials in v.partials, or
// from the state when nd_blocks is 0; |r|^2 partials into v.partials2) and
// its finalize; 1: x += alpha p (unless flushed), p = r + beta p; 2: the FP64
// group's flush of x += alpha p
template <int PA, int PI>
static void launch_blas(const Gauge &gauge, const CgVectors &v, int which, int nd_blocks, hipStream_t s)
{
    const int vh = (int)gauge.vh;
    const int64_t sa = field_bytes(gauge.g, PA, 1), si = field_bytes(gauge.g, PI, 1);
    dim3 grid(blas_blocks(vh), v.nrhs);
    if (which == 0)
        hipLaunchKernelGGL((update_kernel<PA, PI>), grid, dim3(BLAS_BLOCK), 0, s, vh, (char *)v.r, (const char *)v.q,
                           sa, si, v.state, (const double *)v.partials, nd_blocks, v.partials2, v.max_blocks);
    else if (which == 1)
        hipLaunchKernelGGL((pupdate_kernel<PA, PI>), grid, dim3(BLAS_BLOCK), 0, s, vh, (char *)v.xlo,
                           (const char *)v.r, (char *)v.p, sa, si, (const CgState *)v.state);
    else
        hipLaunchKernelGGL((xflush_kernel<PA, PI>), grid, dim3(BLAS_BLOCK), 0, s, vh, (char *)v.xlo,
                           (const char *)v.p, sa, si, (const CgState *)v.state);
    LQS_HIP(hipGetLastError());
    if (which == 0) launch_finalize(v, v.partials2, grid.x, FIN_UPDATE, 0, 0, s);
}

template <int PA, int R, int K>
static void launch_residual_k(const Gauge &gauge, const CgVectors &v, int gate_mode, int mode, hipStream_t s)
{
    const Geom &g = gauge.g;
    const int block = 256;
    const dim3 grid((g.vh + block - 1) / block, (v.nrhs + K - 1) / K);
    const LinkRef L = gauge.ref(F64, R);
    const int lf = (L.temporal ? LF_TEMPORAL : 0) | (default_hop_shape(L, v.nrhs).stream_links ? LF_STREAM : 0);
    const int64_t sa = field_bytes(g, PA, 1);
    char *r = (char *)(mode == 2 ? nullptr : v.r);
#define LQS_RES(LF)                                                                                               \
    hipLaunchKernelGGL((residual_kernel<R, PA, K, LF>), grid, dim3(block), 0, s, g, L, (const char *)v.t64,       \
                       (const char *)v.x, (const char *)v.b, r, sa, v.state, v.partials, v.max_blocks, v.nrhs,  \
                       gate_mode, mode)
    switch (lf) {
    case 0: LQS_RES(0); break;
    case LF_TEMPORAL: LQS_RES(LF_TEMPORAL); break;
    case LF_STREAM: LQS_RES(LF_STREAM); break;
    default: LQS_RES(LF_TEMPORAL | LF_STREAM); break;
    }
#undef LQS_RES
    LQS_HIP(hipGetLastError());
    launch_finalize(v, v.partials, grid.x, FIN_RESID, gate_mode, mode, s);
}

// FP64 residual with the R-real FP64 links (two right-hand sides per thread
// from two on)
static void launch_residual(const Gauge &gauge, const CgVectors &v, int R, int gate_mode, int mode, hipStream_t s)
{
    const bool two = v.nrhs >= 2;
#define LQS_RES_PA(PA)                                                                                            \
    if (R == 12 && two) launch_residual_k<PA, 12, 2>(gauge, v, gate_mode, mode, s);                               \
    else if (R == 12) launch_residual_k<PA, 12, 1>(gauge, v, gate_mode, mode, s);                                 \
    else if (two) launch_residual_k<PA, 18, 2>(gauge, v, gate_mode, mode, s);                                     \
    else launch_residual_k<PA, 18, 1>(gauge, v, gate_mode, mode, s)
    if (v.acc_prec == F64) {
        LQS_RES_PA(F64);
    } else {
        LQS_RES_PA(F32);
    }
#undef LQS_RES_PA
}

static void launch_accumulate(const Gauge &gauge, const CgVectors &v, int gated, hipStream_t s)
{
    const int vh = (int)gauge.vh;
    dim3 grid(blas_blocks(vh), v.nrhs);
    const int64_t sa = field_bytes(gauge.g, v.acc_prec, 1);
    LQS_REQUIRE(v.acc_prec == F32, LQS_EUNSUPPORTED, "accumulate needs an FP32 inner solution");
    hipLaunchKernelGGL((accumulate_kernel<F32>), grid, dim3(BLAS_BLOCK), 0, s, vh, v.x, (char *)v.xlo, sa,
                       (const CgState *)v.state, gated);
    LQS_HIP(hipGetLastError());
}

// t64 = D_oe x and the residual kernel with the R-real FP64 links
static void residual_pass(const Gauge &gauge, const CgVectors &v, int R, int gate_mode, int mode, hipStream_t s)
{
    const LinkRef L64 = gauge.ref(F64, R);
    const LaunchShape sh = default_hop_shape(L64, v.nrhs);
    launch_hop_gated(gauge.g, L64, F64, R, 0, 1, v.nrhs, v.x, v.t64, v.state, gate_mode, sh, s);
    launch_residual(gauge, v, R, gate_mode, mode, s);
}

// The FP64 residual group: x += x_lo (mixed), t64 = D_oe x, residual kernel.
// In a mixed solve on 12-real links the periodic reliable updates use the
// FP64 12-real links (two thirds of the bytes); the update that decides
// convergence always uses the stored 18-real links, so the reported residual
// is that of the operator the caller passed.
void cg_residual_group(Ctx &ctx, const Gauge &gauge, const CgVectors &v, int gate_mode, int mode, hipStream_t s)
{
    (void)ctx;
    const bool mixed = v.acc_prec != F64;
    if (mixed && mode == 0) launch_accumulate(gauge, v, gate_mode == 2 ? 1 : 0, s);
    if (mixed && mode == 0 && gate_mode == 2 && v.recon == 12 && gauge.fmt[F64][1]) {
        residual_pass(gauge, v, 12, 3, 3, s);
        residual_pass(gauge, v, 18, 4, 0, s);
    } else {
        residual_pass(gauge, v, 18, gate_mode, mode, s);
    }
}

void cg_init(Ctx &ctx, const Gauge &gauge, CgVectors &v, bool use_x0, hipStream_t s)
{
    const int vh = (int)gauge.vh;
    dim3 grid(blas_blocks(vh), v.nrhs);
    const int64_t sa = field_bytes(gauge.g, v.acc_prec, 1), si = field_bytes(gauge.g, v.prec, 1);
    char *xlo = v.acc_prec == F64 ? nullptr : (char *)v.xlo;
    const int cold = use_x0 ? 0 : 1;
#define LQS_INIT(PA, PI)                                                                                          \
    hipLaunchKernelGGL((init_kernel<PA, PI>), grid, dim3(BLAS_BLOCK), 0, s, vh, (const char *)v.b, v.x,           \
                       (char *)v.r, (char *)v.p, xlo, sa, si, v.state, v.partials, v.max_blocks, cold)
    if (v.acc_prec == F64) LQS_INIT(F64, F64);
    else if (v.prec == F32) LQS_INIT(F32, F32);
    else LQS_INIT(F32, F16);
#undef LQS_INIT
    LQS_HIP(hipGetLastError());
    launch_finalize(v, v.partials, grid.x, FIN_INIT, 0, cold, s);
    if (use_x0) {
        cg_residual_group(ctx, gauge, v, 0, 1, s);
        launch_convert(gauge.g, v.nrhs, v.acc_prec, v.r, v.prec, v.p, s);
    }
}

// Launch shape of the CG hop (tuned, else the default)
static LaunchShape cg_hop_shape(Ctx &ctx, const Gauge &gauge, int prec, int recon, int nrhs)
{
    LaunchShape sh = default_hop_shape(gauge.ref(prec, recon), nrhs);
    if (ctx.tuner) ctx.tuner->lookup(tune_key(ctx, gauge.temporal ? "hop_tg" : "hop", gauge.g, prec, recon, nrhs), sh);
    return sh;
}

void cg_iteration(Ctx &ctx, const Gauge &gauge, CgVectors &v, hipStream_t s, bool with_reliable)
{
    const LaunchShape sh = cg_hop_shape(ctx, gauge, v.prec, v.recon, v.nrhs);
    LaunchShape shd = default_hop_shape(gauge.ref(v.prec, v.recon), v.nrhs);
    if (ctx.tuner) {
        const bool tg = gauge.temporal;
        ctx.tuner->lookup(tune_key(ctx, tg ? "normal_dot_tg" : "normal_dot", gauge.g, v.prec, v.recon, v.nrhs), shd);
    }
    // 1. t = D_oe p
    prof_begin(ctx, s);
    launch_hop_gated(gauge.g, gauge.ref(v.prec, v.recon), v.prec, v.recon, 0, 1, v.nrhs, v.p, v.t, v.state, 1, sh, s);
    prof_end(ctx, v.prec, v.recon, gauge.vh * v.nrhs, s);
    // 2. q = m^2 p - D_eo t, <p,q>
    launch_normal_dot_shape(gauge, v, shd, s);
    // 3. update
    int nd_blocks = (int)((gauge.vh + shd.block - 1) / shd.block);
    if (nd_blocks > FOLD_ALPHA_MAX) {
        launch_finalize(v, v.partials, nd_blocks, FIN_DOT, 0, 0, s);
        nd_blocks = 0;
    }
    if (v.acc_prec == F64) launch_blas<F64, F64>(gauge, v, 0, nd_blocks, s);
    else if (v.prec == F32) launch_blas<F32, F32>(gauge, v, 0, nd_blocks, s);
    else launch_blas<F32, F16>(gauge, v, 0, nd_blocks, s);
    // FP64 residual group (gated), after the x step it needs
    if (with_reliable) {
        if (v.acc_prec == F64) launch_blas<F64, F64>(gauge, v, 2, 0, s);
        else if (v.prec == F32) launch_blas<F32, F32>(gauge, v, 2, 0, s);
        else launch_blas<F32, F16>(gauge, v, 2, 0, s);
        cg_residual_group(ctx, gauge, v, 2, 0, s);
    }
    // 4. p = r + beta p
    if (v.acc_prec == F64) launch_blas<F64, F64>(gauge, v, 1, 0, s);
    else if (v.prec == F32) launch_blas<F32, F32>(gauge, v, 1, 0, s);
    else launch_blas<F32, F16>(gauge, v, 1, 0, s);
}

// ---------------------------------------------------------------------------
// one problem (nrhs >= 1) with the multi-kernel iteration

static bool final_phase(int32_t ph)
{
    return ph == CG_CONVERGED || ph == CG_BREAKDOWN || ph == CG_NONFINITE || ph == CG_MAXITER;
}

// Initial state records of one problem's right-hand sides.
static void cg_initial_states(const lqs_cg_params &prm, int nrhs, const double *mass, CgState *out)
{
    const bool mixed = prm.inner_prec != F64;
    const int rel_interval = mixed ? (prm.reliable_interval > 0 ? prm.reliable_interval : 100) : 0;
    const double delta =
        mixed ? (prm.reliable_delta > 0 ? prm.reliable_delta : default_reliable_delta(prm.inner_prec)) : 0.0;
    for (int r = 0; r < nrhs; ++r) {
        CgState S{};
        S.stop2 = prm.tol * prm.tol;
        S.delta2 = delta * delta;
        S.rel_interval = rel_interval;
        S.max_iter = prm.max_iter;
        S.phase = CG_RUNNING;
        S.m2 = mass[r] * mass[r];
        out[r] = S;
    }
}

// Device workspace of one problem, every buffer starting on a 256-byte boundary.
size_t cg_workspace_bytes(const Gauge &gauge, const lqs_cg_params &prm, int nrhs)
{
    auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    const bool mixed = prm.inner_prec != F64;
    const size_t fp = field_bytes(gauge.g, prm.inner_prec, nrhs), fa = field_bytes(gauge.g, mixed ? F32 : F64, nrhs),
                 f64 = field_bytes(gauge.g, F64, nrhs);
    const size_t part = sizeof(double) * (size_t)cg_partials_needed(gauge, nrhs) * nrhs;
    size_t n = up(sizeof(CgState) * nrhs) + 2 * up(part) + 3 * up(fp) + up(fa);
    if (mixed) n += up(fa) + up(f64);
    return n;
}

// One problem driven as a small state machine, so that several problems on
// their own streams can be advanced in turn by one host thread.
namespace {

struct CgRun {
    Ctx &ctx;
    lqs_problem pb;
    lqs_cg_params prm;
    lqs_cg_stats *stats;
    hipStream_t s;
    std::string tag;
    std::chrono::steady_clock::time_point t0;
    CgVectors v{};
    bool mixed = false;
    int nrhs = 1;
    size_t sbytes = 0;
    CgState *hs[2] = {nullptr, nullptr};
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipEvent_t tev[2] = {nullptr, nullptr};  // timing: first and last kernel of the solve
    int inflight = 0, slot = 0;
    int64_t enqueued = 0, cap = 0;
    bool done = false;
    bool use_graph = false;  // s is a side stream and graphs are on
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // iterations between FP64 groups (gated launches that return at once unless a
    // reliable update or the final check is pending) and chunks between state polls
    static constexpr int chunk = 8;
    static constexpr int poll_every = 1;

    CgRun(Ctx &c, const lqs_problem &p, const lqs_cg_params &pr, lqs_cg_stats *st, hipStream_t str, std::string tg,
          std::chrono::steady_clock::time_point start)
        : ctx(c), pb(p), prm(pr), stats(st), s(str), tag(std::move(tg)), t0(start)
    {
    }
    ~CgRun()
    {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
        for (hipEvent_t e : tev)
            if (e) (void)hipEventDestroy(e);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }

    // one round: poll_every chunks of iterations, each closed by the gated FP64 group
    void round()
    {
        for (int c = 0; c < poll_every; ++c)
            for (int i = 0; i < chunk; ++i) cg_iteration(ctx, gauge(), v, s, i == chunk - 1);
    }
    const Gauge &gauge() const { return *pb.gauge; }

    // Buffers come from the context's workspace, or, when `arena` is set,
    // are carved from that preallocated device region (no allocation).
    std::vector<double> masses;  // per right-hand side (empty: pb.mass for all)
    char *arena = nullptr;
    size_t arena_bytes = 0, arena_used = 0;
    CgState *arena_host = nullptr;  // host mirror (two records per rhs) with an arena
    void *buf(const std::string &slot, size_t bytes)
    {
        if (!arena) return ctx.workspace(slot + tag, bytes);
        const size_t off = (arena_used + 255) & ~size_t(255);
        LQS_REQUIRE(off + bytes <= arena_bytes, LQS_EINVAL, "workspace exceeds the preallocated region");
        arena_used = off + bytes;
        return arena + off;
    }

    void setup()
    {
        const Geom &g = gauge().g;
        nrhs = pb.nrhs;
        mixed = prm.inner_prec != F64;
        v.prec = prm.inner_prec;
        v.acc_prec = mixed ? F32 : F64;
        v.recon = prm.inner_recon == 12 ? 12 : 18;
        v.nrhs = nrhs;
        v.mass = pb.mass;
        (void)gauge().ref(v.prec, v.recon);  // format must exist
        v.max_blocks = cg_partials_needed(gauge(), nrhs);
        sbytes = sizeof(CgState) * nrhs;
        // every size is checked before the first launch
        const size_t need = cg_workspace_bytes(gauge(), prm, nrhs);
        LQS_REQUIRE(!arena || need <= arena_bytes, LQS_EINVAL,
                    "solve needs " + std::to_string(need) + " bytes of workspace, the preallocated region holds " +
                        std::to_string(arena_bytes));
        const int64_t fp = field_bytes(g, v.prec, nrhs), fa = field_bytes(g, v.acc_prec, nrhs),
                      f64 = field_bytes(g, F64, nrhs);
        v.state = (CgState *)buf("cg.state", sbytes);
        v.partials = (double *)buf("cg.partials", sizeof(double) * (size_t)v.max_blocks * nrhs);
        v.partials2 = (double *)buf("cg.partials2", sizeof(double) * (size_t)v.max_blocks * nrhs);
        v.p = buf("cg.p", fp);
        v.q = buf("cg.q", fp);
        v.t = buf("cg.t", fp);
        v.x = pb.x;
        v.b = (double *)pb.b;
        if (mixed) {
            v.r = buf("cg.r", fa);
            v.xlo = buf("cg.xlo", fa);
            v.t64 = buf("cg.t64", f64);
            v.rhi = nullptr;
        } else {
            v.r = buf("cg.r", f64);
            v.xlo = pb.x;
            v.t64 = v.t;
            v.rhi = (double *)v.r;
        }
        if (arena) {
            hs[0] = arena_host;
            hs[1] = arena_host + nrhs;
        } else {
            char *host = (char *)ctx.pinned("cg.host" + tag, 2 * sbytes);
            hs[0] = (CgState *)host;
            hs[1] = (CgState *)(host + sbytes);
        }
        std::vector<double> mass(nrhs, pb.mass);
        if (!masses.empty()) mass = masses;
        LQS_REQUIRE((int)mass.size() == nrhs, LQS_EINVAL, "one mass per right-hand side");
        cg_initial_states(prm, nrhs, mass.data(), hs[0]);
        if (!arena) {
            LQS_HIP(hipEventCreate(&tev[0]));
            LQS_HIP(hipEventCreate(&tev[1]));
            LQS_HIP(hipEventRecord(tev[0], s));
        }
        LQS_HIP(hipMemcpyAsync(v.state, hs[0], sbytes, hipMemcpyHostToDevice, s));
        cg_init(ctx, gauge(), v, prm.use_x0 != 0, s);
        if (!arena) {
            LQS_HIP(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
            LQS_HIP(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
        }
        cap = (int64_t)prm.max_iter + 16 * chunk + 64;
    }

    // queue one round of iterations and an asynchronous poll of the state.
    // With graphs the round is captured once (the kernels read their scalars
    // and gates from the device state, so every replay is the same work) and
    // replayed; the round holds no memset or host synchronisation.
    void enqueue()
    {
        if (use_graph) {
            if (!exec) {
                LQS_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
                try {
                    round();
                } catch (...) {
                    hipGraph_t g = nullptr;
                    (void)hipStreamEndCapture(s, &g);
                    if (g) (void)hipGraphDestroy(g);
                    throw;
                }
                LQS_HIP(hipStreamEndCapture(s, &graph));
                LQS_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
            }
            LQS_HIP(hipGraphLaunch(exec, s));
        } else {
            round();
        }
        enqueued += chunk * poll_every;
        LQS_HIP(hipMemcpyAsync(hs[slot], v.state, sbytes, hipMemcpyDeviceToHost, s));
        if (arena) {
            // no events: wait for this poll at once
            LQS_HIP(hipStreamSynchronize(s));
            decide(hs[slot]);
            return;
        }
        LQS_HIP(hipEventRecord(ev[slot], s));
        ++inflight;
        slot ^= 1;
    }

    void decide(const CgState *h)
    {
        bool all = true;
        for (int r = 0; r < nrhs; ++r) all &= final_phase(h[r].phase);
        if (all || enqueued > cap) done = true;
    }

    // with two polls in flight, wait for the older one and decide
    void check()
    {
        if (inflight < 2) return;
        LQS_HIP(hipEventSynchronize(ev[slot]));
        --inflight;
        decide(hs[slot]);
    }

    void finish()
    {
        LQS_HIP(hipStreamSynchronize(s));
        // right-hand sides that stopped without an FP64 check (breakdown,
        // non-finite, host cap) get x += x_lo and a measured residual
        LQS_HIP(hipMemcpyAsync(hs[0], v.state, sbytes, hipMemcpyDeviceToHost, s));
        LQS_HIP(hipStreamSynchronize(s));
        bool need = false;
        for (int r = 0; r < nrhs; ++r) need |= !(hs[0][r].phase == CG_CONVERGED || hs[0][r].phase == CG_MAXITER);
        if (need) {
            if (mixed) launch_accumulate(gauge(), v, 0, s);
            cg_residual_group(ctx, gauge(), v, 0, 2, s);
            LQS_HIP(hipMemcpyAsync(hs[0], v.state, sbytes, hipMemcpyDeviceToHost, s));
            LQS_HIP(hipStreamSynchronize(s));
        }
        float dev_ms = 0.f;
        if (tev[0]) {
            LQS_HIP(hipEventRecord(tev[1], s));
            LQS_HIP(hipEventSynchronize(tev[1]));
            LQS_HIP(hipEventElapsedTime(&dev_ms, tev[0], tev[1]));
        }
        const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        for (int r = 0; r < nrhs; ++r) {
            const CgState &S = hs[0][r];
            lqs_cg_stats &o = stats[r];
            o.iters = S.iters;
            o.reliable_updates = S.nreliable;
            o.restarts = S.restarts;
            o.true_rel_residual = S.b2 > 0 ? std::sqrt(S.true_r2 / S.b2) : 0.0;
            o.seconds = secs;
            o.device_seconds = 1e-3 * dev_ms;
            cg_fill_rates(o, gauge(), v.prec, v.recon, nrhs);
            switch (S.phase) {
            case CG_CONVERGED: o.status = LQS_OK; break;
            case CG_BREAKDOWN: o.status = LQS_EBREAKDOWN; break;
            case CG_NONFINITE: o.status = LQS_ENONFINITE; break;
            default: o.status = LQS_ENOTCONV; break;
            }
        }
    }
};

}  // namespace

void cg_solve_one(Ctx &ctx, const lqs_problem &pb, const lqs_cg_params &prm, lqs_cg_stats *stats, hipStream_t s,
                  const std::vector<double> *masses)
{
    // graphs are captured on a side stream (the caller's stream may be the
    // null stream, which cannot be captured), forked from and joined into s
    const bool graphs = ctx.graphs && !ctx.profiling;
    hipStream_t rs = graphs ? ctx.side_stream(0) : s;
    hipEvent_t fork = nullptr, join = nullptr;
    if (graphs) {
        LQS_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
        LQS_HIP(hipEventCreateWithFlags(&join, hipEventDisableTiming));
    }
    auto cleanup = [&]() {
        if (fork) (void)hipEventDestroy(fork);
        if (join) (void)hipEventDestroy(join);
    };
    try {
        if (graphs) {
            LQS_HIP(hipEventRecord(fork, s));
            LQS_HIP(hipStreamWaitEvent(rs, fork, 0));
        }
        CgRun run(ctx, pb, prm, stats, rs, "", std::chrono::steady_clock::now());
        run.use_graph = graphs;
        if (masses) run.masses = *masses;
        run.setup();
        try {
            while (!run.done) {
                run.enqueue();
                run.check();
            }
        } catch (...) {
            (void)hipStreamSynchronize(rs);
            throw;
        }
        run.finish();
        if (graphs) {
            LQS_HIP(hipEventRecord(join, rs));
            LQS_HIP(hipStreamWaitEvent(s, join, 0));
        }
    } catch (...) {
        cleanup();
        throw;
    }
    cleanup();
}

// Problems of different sizes each get a side stream (forked from and joined
// back into s with events) and their own workspaces; the host enqueues a
// round of iterations for every unfinished problem before it waits on any
// poll, so the small lattices' kernels fill the gaps of the large ones.
void cg_solve_concurrent(Ctx &ctx, int nprob, const lqs_problem *probs, const lqs_cg_params &prm,
                         lqs_cg_stats *stats, hipStream_t s)
{
    constexpr int MAX_SIDE = 8;
    const auto t0 = std::chrono::steady_clock::now();
    const int nside = nprob < MAX_SIDE ? nprob : MAX_SIDE;
    hipEvent_t fork = nullptr;
    LQS_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    std::vector<hipEvent_t> joins;
    std::vector<std::unique_ptr<CgRun>> runs;
    auto cleanup = [&]() {
        for (int k = 0; k < nside; ++k) (void)hipStreamSynchronize(ctx.side_stream(k));
        for (hipEvent_t e : joins) (void)hipEventDestroy(e);
        (void)hipEventDestroy(fork);
    };
    try {
        LQS_HIP(hipEventRecord(fork, s));
        for (int k = 0; k < nside; ++k) LQS_HIP(hipStreamWaitEvent(ctx.side_stream(k), fork, 0));
        int off = 0;
        for (int i = 0; i < nprob; ++i) {
            runs.emplace_back(new CgRun(ctx, probs[i], prm, stats + off, ctx.side_stream(i % nside),
                                        "#" + std::to_string(i), t0));
            runs.back()->use_graph = ctx.graphs && !ctx.profiling;
            off += probs[i].nrhs;
        }
        for (auto &r : runs) r->setup();
        bool any = true;
        while (any) {
            any = false;
            for (auto &r : runs)
                if (!r->done) r->enqueue();
            for (auto &r : runs)
                if (!r->done) {
                    r->check();
                    any |= !r->done;
                }
        }
        for (auto &r : runs) r->finish();
        for (int k = 0; k < nside; ++k) {
            hipEvent_t e = nullptr;
            LQS_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            joins.push_back(e);
            LQS_HIP(hipEventRecord(e, ctx.side_stream(k)));
            LQS_HIP(hipStreamWaitEvent(s, e, 0));
        }
    } catch (...) {
        cleanup();
        throw;
    }
    cleanup();
}


// ---------------------------------------------------------------------------
// A solve that allocates nothing, for callers that cannot allocate device
// memory.  Its workspace is a file-scope device array (each GPU the library
// runs on holds its own copy until the process ends); host code never uses
// the array's name as an address, only the per-device address fetched once
// with hipGetSymbolAddress.  Every call on one GPU shares that GPU's array:
// calls that overlap on one GPU race.  The solve runs eagerly on the caller's
// stream (no graphs, no events, no pinned host buffers), with the kernels of
// cg_solve and the same launch shapes.

static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

static std::mutex scratch_mu;
static void *scratch_ptr[NOALLOC_MAX_DEVICES];

// Device address of this GPU's scratch array; the device must be current.
void *noalloc_scratch(int device)
{
    LQS_REQUIRE(device >= 0 && device < NOALLOC_MAX_DEVICES, LQS_EUNSUPPORTED, "device index too large");
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[device]) {
        void *ptr = nullptr;
        LQS_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        scratch_ptr[device] = ptr;
    }
    return scratch_ptr[device];
}

void cg_solve_noalloc_impl(Ctx &ctx, const lqs_problem &pb, const lqs_cg_params &prm, lqs_cg_stats *stats,
                           hipStream_t s)
{
    LQS_REQUIRE(ctx.noalloc_scratch != nullptr, LQS_EHIP, "scratch address not set up");
    const size_t need = cg_workspace_bytes(*pb.gauge, prm, pb.nrhs);
    LQS_REQUIRE(need <= NOALLOC_SCRATCH_BYTES, LQS_EINVAL,
                "solve needs " + std::to_string(need) + " bytes of workspace, more than the " +
                    std::to_string(NOALLOC_SCRATCH_BYTES) + "-byte scratch array");
    // hop profiling records events it creates on demand: off for this call
    struct ProfOff {
        Ctx &c;
        bool was;
        ~ProfOff() { c.profiling = was; }
    } prof{ctx, ctx.profiling};
    ctx.profiling = false;
    CgState host[2 * 16];
    CgRun run(ctx, pb, prm, stats, s, "", std::chrono::steady_clock::now());
    run.arena = (char *)ctx.noalloc_scratch;
    run.arena_bytes = NOALLOC_SCRATCH_BYTES;
    run.arena_host = host;
    try {
        run.setup();
        while (!run.done) run.enqueue();
    } catch (...) {
        (void)hipStreamSynchronize(s);
        throw;
    }
    run.finish();
}

}  // namespace lqs
