// persistent.hip -- several independent even-odd CG solves (lattices of any
// size, each with its own links, mass and source) in ONE cooperative launch.
//
// Small lattices spend most of a multi-kernel CG iteration in launch gaps and
// global reductions (the latency the paper blames for the gap between its
// Dslash and CG numbers, Sec. 4.2).  Here every block stays resident and
// walks a combined tile list (tile = blockDim.x consecutive sites of one
// lattice); the phases of an iteration are separated by grid barriers:
//   hop t = D_oe p | q = m^2 p - D_eo t, tile partials of <p,q>
//   | alpha per lattice; x_lo += alpha p, r -= alpha q, tile partials of |r|^2
//   | beta, stop and reliable-update decisions | [FP64 residual group] p = r + beta p |
// Each block sums the tile partials of every lattice itself in a fixed order,
// so every block holds bit-identical per-lattice scalars and takes the same
// branches without another barrier.  A lattice that has converged is skipped
// by all phases.  The grid barrier waits with a bounded spin; on timeout it
// raises an abort flag that ends every block's loop.
#include <chrono>
#include <cmath>

#include "hop.hpp"

namespace lqs {

static constexpr int PMAX_LAT = 8;
static constexpr int PBLOCK = 256;

struct PLat {
    Geom g;
    LinkRef lo, hi;
    double m2;
    char *p, *q, *t, *r, *xlo, *t64;
    double *x;
    const double *b;
    int tile0, ntiles;
    double *part[2];    // tile partials, two buffers used alternately
};

struct GridBar {
    uint32_t count;
    uint32_t gen;
    uint32_t abort;
    uint32_t pad;
};

// Grid barrier.  On this GPU every XCD has its own L2, so making a block's
// stores visible to blocks on other XCDs takes an agent-scope release (an L2
// write-back) and reading theirs an agent-scope acquire (an L2 invalidate).
// Each block pays exactly one of each per barrier: thread 0 releases, arrives
// with a relaxed atomic, spins with relaxed loads (no cache maintenance per
// poll), then acquires.  The last block to arrive resets the counter before
// it publishes the new generation with a release store, so no block can
// arrive at the next barrier before the reset is visible.
__device__ __forceinline__ bool grid_sync(GridBar *gb, uint32_t nblocks, uint32_t &gen)
{
    __shared__ uint32_t aborted;
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const uint32_t old = __hip_atomic_fetch_add(&gb->count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (old == nblocks - 1) {
            __hip_atomic_store(&gb->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&gb->gen, gen + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            uint32_t spins = 0;
            while (__hip_atomic_load(&gb->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > (1u << 22)) {
                    __hip_atomic_store(&gb->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                if ((spins & 255) == 0 && __hip_atomic_load(&gb->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                    break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        gen += 1;
        aborted = __hip_atomic_load(&gb->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    return aborted == 0;
}

__device__ __forceinline__ int lattice_of(const PLat *L, int nlat, int tile)
{
    int l = 0;
    while (l + 1 < nlat && tile >= L[l + 1].tile0) ++l;
    return l;
}

__device__ void p_fin_update(CgState &S, double r2)
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

__device__ void p_fin_residual(CgState &S, double r2)
{
    S.true_r2 = r2;
    S.nreliable += 1;
    S.reliable_pending = 0;
    S.since_rel = 0;
    if (!isfinite(r2)) S.phase = CG_NONFINITE;
    else if (r2 <= S.stop2) S.phase = CG_CONVERGED;
    else if (S.iters >= S.max_iter) S.phase = CG_MAXITER;
    else {
        if (S.rel_interval == 0) {
            S.beta = 0.0;
            S.restarts += 1;
        } else {
            S.beta = r2 / S.rho_old;
        }
        S.rho = r2;
        S.max_rho = r2;
        S.phase = CG_RUNNING;
    }
}

template <int P, int R, int PA>
__global__ void __launch_bounds__(PBLOCK) persistent_cg_kernel(const PLat *lats, int nlat, int ntiles, CgState *st_out,
                                                               GridBar *gb, int max_trips)
{
    typedef typename RealOf<P>::type T;
    typedef typename RealOf<PA>::type TA;
    __shared__ CgState S[PMAX_LAT];
    __shared__ PLat D[PMAX_LAT];
    __shared__ int any_running, any_pending;
    uint32_t gen = 0;
    const uint32_t nb = gridDim.x;
    if (threadIdx.x < nlat) {
        S[threadIdx.x] = st_out[threadIdx.x];
        D[threadIdx.x] = lats[threadIdx.x];
    }
    __syncthreads();

    // ---- cold start: x = x_lo = 0, r = p = b, tile partials of |b|^2
    for (int tile = blockIdx.x; tile < ntiles; tile += nb) {
        const int l = lattice_of(D, nlat, tile);
        const PLat &L = D[l];
        const int cb = (tile - L.tile0) * PBLOCK + threadIdx.x;
        double loc = 0.0;
        if (cb < L.g.vh) {
            const V3<double> bv = SpinorIO<F64>::load(L.b, L.g.vh, cb);
#pragma unroll
            for (int a = 0; a < 3; ++a) loc += bv.c[a].re * bv.c[a].re + bv.c[a].im * bv.c[a].im;
            SpinorIO<F64>::store(L.x, L.g.vh, cb, vzero<double>());
            SpinorIO<PA>::store(L.xlo, L.g.vh, cb, vzero<TA>());
            SpinorIO<PA>::store(L.r, L.g.vh, cb, vcast<TA>(bv));
            SpinorIO<P>::store(L.p, L.g.vh, cb, vcast<T>(bv));
        }
        const double s = block_sum(loc);
        if (threadIdx.x == 0) L.part[0][tile - L.tile0] = s;
    }
    if (!grid_sync(gb, nb, gen)) goto out;
    for (int l = 0; l < nlat; ++l) {
        const double b2 = sum_partials(D[l].part[0], D[l].ntiles);
        if (threadIdx.x == 0) {
            S[l].b2 = b2;
            S[l].stop2 *= b2;
            S[l].rho = b2;
            S[l].max_rho = b2;
            S[l].true_r2 = b2;
            S[l].phase = (b2 == 0.0) ? CG_CONVERGED : (isfinite(b2) ? CG_RUNNING : CG_NONFINITE);
        }
    }
    __syncthreads();

    for (int trip = 0; trip < max_trips; ++trip) {
        if (threadIdx.x == 0) {
            int a = 0;
            for (int l = 0; l < nlat; ++l) a |= (S[l].phase == CG_RUNNING);
            any_running = a;
        }
        __syncthreads();
        if (!any_running) break;

        // ---- t = D_oe p
        for (int tile = blockIdx.x; tile < ntiles; tile += nb) {
            const int l = lattice_of(D, nlat, tile);
            if (S[l].phase != CG_RUNNING) continue;
            const PLat &L = D[l];
            const int cb = (tile - L.tile0) * PBLOCK + threadIdx.x;
            if (cb >= L.g.vh) continue;
            const Site s = decode(L.g, cb, 1);
            V3<T> acc;
            const bool act = true;
            hop_site<P, R, 1>(L.g, L.lo, 1, s, cb, L.p, 0, &act, &acc);
            SpinorIO<P>::store(L.t, L.g.vh, cb, acc);
        }
        if (!grid_sync(gb, nb, gen)) break;

        // ---- q = m^2 p - D_eo t, tile partials of <p, q>
        for (int tile = blockIdx.x; tile < ntiles; tile += nb) {
            const int l = lattice_of(D, nlat, tile);
            if (S[l].phase != CG_RUNNING) continue;
            const PLat &L = D[l];
            const int cb = (tile - L.tile0) * PBLOCK + threadIdx.x;
            double dot = 0.0;
            if (cb < L.g.vh) {
                const Site s = decode(L.g, cb, 0);
                V3<T> acc;
                const bool act = true;
                hop_site<P, R, 1>(L.g, L.lo, 0, s, cb, L.t, 0, &act, &acc);
                const V3<T> pv = SpinorIO<P>::load(L.p, L.g.vh, cb);
                V3<T> qv;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    qv.c[a].re = (T)L.m2 * pv.c[a].re - acc.c[a].re;
                    qv.c[a].im = (T)L.m2 * pv.c[a].im - acc.c[a].im;
                    dot += (double)pv.c[a].re * (double)qv.c[a].re + (double)pv.c[a].im * (double)qv.c[a].im;
                }
                SpinorIO<P>::store(L.q, L.g.vh, cb, qv);
            }
            const double s = block_sum(dot);
            if (threadIdx.x == 0) L.part[0][tile - L.tile0] = s;
        }
        if (!grid_sync(gb, nb, gen)) break;
        for (int l = 0; l < nlat; ++l) {
            if (S[l].phase != CG_RUNNING) continue;
            const double pq = sum_partials(D[l].part[0], D[l].ntiles);
            if (threadIdx.x == 0) {
                if (!isfinite(pq)) S[l].phase = CG_NONFINITE;
                else if (!(pq > 0.0)) S[l].phase = CG_BREAKDOWN;
                else S[l].alpha = S[l].rho / pq;
            }
            __syncthreads();
        }
        // The update below writes the other partial buffer, so no barrier is
        // needed between these reads and those writes; buffer 0 is written
        // again only after at least two more barriers.

        // ---- x_lo += alpha p, r -= alpha q, tile partials of |r|^2
        for (int tile = blockIdx.x; tile < ntiles; tile += nb) {
            const int l = lattice_of(D, nlat, tile);
            if (S[l].phase != CG_RUNNING) continue;
            const PLat &L = D[l];
            const int cb = (tile - L.tile0) * PBLOCK + threadIdx.x;
            double loc = 0.0;
            if (cb < L.g.vh) {
                const TA alpha = (TA)S[l].alpha;
                const V3<TA> pv = vcast<TA>(SpinorIO<P>::load(L.p, L.g.vh, cb));
                const V3<TA> qv = vcast<TA>(SpinorIO<P>::load(L.q, L.g.vh, cb));
                V3<TA> xv = SpinorIO<PA>::load(L.xlo, L.g.vh, cb);
                V3<TA> rv = SpinorIO<PA>::load(L.r, L.g.vh, cb);
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    xv.c[a].re += alpha * pv.c[a].re;
                    xv.c[a].im += alpha * pv.c[a].im;
                    rv.c[a].re -= alpha * qv.c[a].re;
                    rv.c[a].im -= alpha * qv.c[a].im;
                    loc += (double)rv.c[a].re * (double)rv.c[a].re + (double)rv.c[a].im * (double)rv.c[a].im;
                }
                SpinorIO<PA>::store(L.xlo, L.g.vh, cb, xv);
                SpinorIO<PA>::store(L.r, L.g.vh, cb, rv);
            }
            const double s = block_sum(loc);
            if (threadIdx.x == 0) L.part[1][tile - L.tile0] = s;
        }
        if (!grid_sync(gb, nb, gen)) break;
        for (int l = 0; l < nlat; ++l) {
            if (S[l].phase != CG_RUNNING) continue;
            const double r2 = sum_partials(D[l].part[1], D[l].ntiles);
            if (threadIdx.x == 0) p_fin_update(S[l], r2);
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            int a = 0;
            for (int l = 0; l < nlat; ++l) a |= S[l].reliable_pending;
            any_pending = a;
        }
        __syncthreads();

        if (any_pending) {
            // ---- t64 = D_oe (x + x_lo) in FP64
            for (int tile = blockIdx.x; tile < ntiles; tile += nb) {
                const int l = lattice_of(D, nlat, tile);
                if (!S[l].reliable_pending) continue;
                const PLat &L = D[l];
                const int cb = (tile - L.tile0) * PBLOCK + threadIdx.x;
                if (cb >= L.g.vh) continue;
                const Site s = decode(L.g, cb, 1);
                V3<double> acc = vzero<double>();
                const char *lb = (const char *)L.hi.base;
#pragma unroll
                for (int mu = 0; mu < 4; ++mu) {
                    const M3<double> uf = LinkIO<F64, 18>::load(lb + (2 * mu + 1) * L.hi.block_bytes, L.g.vh, cb);
                    V3<double> v = SpinorIO<F64>::load(L.x, L.g.vh, s.fwd[mu]);
                    V3<double> w = vcast<double>(SpinorIO<PA>::load(L.xlo, L.g.vh, s.fwd[mu]));
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        v.c[a].re += w.c[a].re;
                        v.c[a].im += w.c[a].im;
                    }
                    accum(acc, mv(uf, v), (s.negf >> mu) & 1);
                    const M3<double> ub = LinkIO<F64, 18>::load(lb + (2 * mu) * L.hi.block_bytes, L.g.vh, s.bwd[mu]);
                    v = SpinorIO<F64>::load(L.x, L.g.vh, s.bwd[mu]);
                    w = vcast<double>(SpinorIO<PA>::load(L.xlo, L.g.vh, s.bwd[mu]));
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        v.c[a].re += w.c[a].re;
                        v.c[a].im += w.c[a].im;
                    }
                    accum(acc, mdv(ub, v), !((s.negb >> mu) & 1));
                }
                SpinorIO<F64>::store(L.t64, L.g.vh, cb, acc);
            }
            if (!grid_sync(gb, nb, gen)) break;
            // ---- x += x_lo, x_lo = 0, r_hi = b - (m^2 x - D_eo t64), r = r_hi
            for (int tile = blockIdx.x; tile < ntiles; tile += nb) {
                const int l = lattice_of(D, nlat, tile);
                if (!S[l].reliable_pending) continue;
                const PLat &L = D[l];
                const int cb = (tile - L.tile0) * PBLOCK + threadIdx.x;
                double loc = 0.0;
                if (cb < L.g.vh) {
                    const Site s = decode(L.g, cb, 0);
                    V3<double> acc;
                    const bool act = true;
                    hop_site<F64, 18, 1>(L.g, L.hi, 0, s, cb, L.t64, 0, &act, &acc);
                    V3<double> xv = SpinorIO<F64>::load(L.x, L.g.vh, cb);
                    const V3<double> lv = vcast<double>(SpinorIO<PA>::load(L.xlo, L.g.vh, cb));
                    const V3<double> bv = SpinorIO<F64>::load(L.b, L.g.vh, cb);
                    V3<double> rv;
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        xv.c[a].re += lv.c[a].re;
                        xv.c[a].im += lv.c[a].im;
                        rv.c[a].re = bv.c[a].re - (L.m2 * xv.c[a].re - acc.c[a].re);
                        rv.c[a].im = bv.c[a].im - (L.m2 * xv.c[a].im - acc.c[a].im);
                        loc += rv.c[a].re * rv.c[a].re + rv.c[a].im * rv.c[a].im;
                    }
                    SpinorIO<F64>::store(L.x, L.g.vh, cb, xv);
                    SpinorIO<PA>::store(L.xlo, L.g.vh, cb, vzero<TA>());
                    SpinorIO<PA>::store(L.r, L.g.vh, cb, vcast<TA>(rv));
                }
                const double s = block_sum(loc);
                if (threadIdx.x == 0) L.part[0][tile - L.tile0] = s;
            }
            if (!grid_sync(gb, nb, gen)) break;
            for (int l = 0; l < nlat; ++l) {
                if (!S[l].reliable_pending) continue;
                const double r2 = sum_partials(D[l].part[0], D[l].ntiles);
                if (threadIdx.x == 0) p_fin_residual(S[l], r2);
                __syncthreads();
            }
        }

        // ---- p = r + beta p
        for (int tile = blockIdx.x; tile < ntiles; tile += nb) {
            const int l = lattice_of(D, nlat, tile);
            if (S[l].phase != CG_RUNNING) continue;
            const PLat &L = D[l];
            const int cb = (tile - L.tile0) * PBLOCK + threadIdx.x;
            if (cb >= L.g.vh) continue;
            const TA beta = (TA)S[l].beta;
            const V3<TA> rv = SpinorIO<PA>::load(L.r, L.g.vh, cb);
            const V3<TA> pv = vcast<TA>(SpinorIO<P>::load(L.p, L.g.vh, cb));
            V3<TA> o;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                o.c[a].re = rv.c[a].re + beta * pv.c[a].re;
                o.c[a].im = rv.c[a].im + beta * pv.c[a].im;
            }
            SpinorIO<P>::store(L.p, L.g.vh, cb, vcast<T>(o));
        }
        if (!grid_sync(gb, nb, gen)) break;
    }
out:
    if (blockIdx.x == 0 && threadIdx.x < nlat) st_out[threadIdx.x] = S[threadIdx.x];
}

// ---------------------------------------------------------------------------

template <int P, int R, int PA> static const void *kernel_ptr() { return (const void *)&persistent_cg_kernel<P, R, PA>; }

static const void *pick_kernel(int prec, int recon)
{
    if (prec == F64) return recon == 12 ? kernel_ptr<F64, 12, F64>() : kernel_ptr<F64, 18, F64>();
    if (prec == F32) return recon == 12 ? kernel_ptr<F32, 12, F32>() : kernel_ptr<F32, 18, F32>();
    return recon == 12 ? kernel_ptr<F16, 12, F32>() : kernel_ptr<F16, 18, F32>();
}

void persistent_solve(Ctx &ctx, const std::vector<PersistentProblem> &probs, const lqs_cg_params &prm,
                      lqs_cg_stats *stats, hipStream_t s)
{
    auto t0 = std::chrono::steady_clock::now();
    const int nlat = (int)probs.size();
    LQS_REQUIRE(nlat >= 1 && nlat <= PMAX_LAT, LQS_EUNSUPPORTED, "persistent solve takes 1..8 lattices");
    LQS_REQUIRE(!prm.use_x0, LQS_EUNSUPPORTED, "persistent solve starts from x = 0");
    int coop = 0;
    LQS_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, ctx.device));
    LQS_REQUIRE(coop, LQS_EUNSUPPORTED, "device has no cooperative launch");
    const int prec = prm.inner_prec, recon = prm.inner_recon == 12 ? 12 : 18;
    const int pa = prec == F64 ? F64 : F32;
    const bool mixed = prec != F64;

    std::vector<PLat> L(nlat);
    int tiles = 0;
    size_t part_total = 0;
    for (int l = 0; l < nlat; ++l) {
        const Gauge &gg = *probs[l].gauge;
        const int nt = (int)((gg.vh + PBLOCK - 1) / PBLOCK);
        L[l].tile0 = tiles;
        L[l].ntiles = nt;
        tiles += nt;
        part_total += nt;
    }
    double *partials = (double *)ctx.workspace("pcg.partials", 2 * sizeof(double) * part_total);
    size_t off = 0;
    for (int l = 0; l < nlat; ++l) {
        const Gauge &gg = *probs[l].gauge;
        PLat &d = L[l];
        d.g = gg.g;
        d.lo = gg.ref(prec, recon);
        d.hi = gg.ref(F64, 18);
        d.m2 = probs[l].mass * probs[l].mass;
        const std::string k = "pcg." + std::to_string(l) + ".";
        const int64_t fp = field_bytes(gg.g, prec, 1), fa = field_bytes(gg.g, pa, 1), f64 = field_bytes(gg.g, F64, 1);
        d.p = (char *)ctx.workspace(k + "p", fp);
        d.q = (char *)ctx.workspace(k + "q", fp);
        d.t = (char *)ctx.workspace(k + "t", fp);
        d.r = (char *)ctx.workspace(k + "r", fa);
        d.xlo = (char *)ctx.workspace(k + "xlo", fa);
        d.t64 = (char *)ctx.workspace(k + "t64", f64);
        d.x = probs[l].x;
        d.b = probs[l].b;
        d.part[0] = partials + off;
        d.part[1] = partials + part_total + off;
        off += d.ntiles;
    }
    PLat *dL = (PLat *)ctx.workspace("pcg.desc", sizeof(PLat) * nlat);
    CgState *dS = (CgState *)ctx.workspace("pcg.state", sizeof(CgState) * nlat);
    GridBar *gb = (GridBar *)ctx.workspace("pcg.bar", sizeof(GridBar));
    std::vector<CgState> hs(nlat);
    const int rel_interval = mixed ? (prm.reliable_interval > 0 ? prm.reliable_interval : 100) : 0;
    const double delta = mixed ? (prm.reliable_delta > 0 ? prm.reliable_delta : 0.1) : 0.0;
    for (auto &S : hs) {
        S = CgState{};
        S.stop2 = prm.tol * prm.tol;
        S.delta2 = delta * delta;
        S.rel_interval = rel_interval;
        S.max_iter = prm.max_iter;
        S.phase = CG_RUNNING;
    }
    LQS_HIP(hipMemcpyAsync(dL, L.data(), sizeof(PLat) * nlat, hipMemcpyHostToDevice, s));

    const void *fn = pick_kernel(prec, recon);
    int per_cu = 0;
    LQS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, PBLOCK, 0));
    LQS_REQUIRE(per_cu >= 1, LQS_EUNSUPPORTED, "persistent kernel does not fit on a compute unit");
    const int max_trips = prm.max_iter + 8;
    int ntiles = tiles;
    const std::vector<CgState> init = hs;
    GridBar hb{};
    // One complete solve with `bpc` resident blocks per compute unit.
    auto solve_once = [&](int bpc) {
        int grid = std::min(bpc, per_cu) * ctx.num_cu;
        if (grid > tiles) grid = tiles;
        LQS_HIP(hipMemcpyAsync(dS, init.data(), sizeof(CgState) * nlat, hipMemcpyHostToDevice, s));
        LQS_HIP(hipMemsetAsync(gb, 0, sizeof(GridBar), s));
        void *args[] = {(void *)&dL, (void *)&nlat, (void *)&ntiles, (void *)&dS, (void *)&gb, (void *)&max_trips};
        LQS_HIP(hipLaunchCooperativeKernel(fn, dim3(grid), dim3(PBLOCK), args, 0, s));
        LQS_HIP(hipMemcpyAsync(hs.data(), dS, sizeof(CgState) * nlat, hipMemcpyDeviceToHost, s));
        LQS_HIP(hipMemcpyAsync(&hb, gb, sizeof(GridBar), hipMemcpyDeviceToHost, s));
        LQS_HIP(hipStreamSynchronize(s));
        LQS_REQUIRE(hb.abort == 0, LQS_EHIP, "persistent solve: grid barrier timed out");
    };
    // The tuned value is the number of resident blocks per compute unit
    // (stored as block = 64 * bpc); the key names every lattice of the batch.
    std::string key = std::string(ctx.prop.gcnArchName) + "|persistent|p" + std::to_string(prec) + "|r" +
                      std::to_string(recon);
    for (const PLat &d : L)
        key += "|" + std::to_string(d.g.n[0]) + "x" + std::to_string(d.g.n[1]) + "x" + std::to_string(d.g.n[2]) +
               "x" + std::to_string(d.g.n[3]);
    int bpc = 2;
    LaunchShape t;
    if (ctx.tuner && ctx.tuner->lookup(key, t)) {
        bpc = t.block / 64;
    } else if (ctx.tuning && ctx.tuner) {
        double best = 1e30;
        for (int c : {1, 2, 4, 8}) {
            if (c > per_cu) break;
            auto a0 = std::chrono::steady_clock::now();
            solve_once(c);
            const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - a0).count();
            if (dt < best) {
                best = dt;
                bpc = c;
            }
        }
        ctx.tuner->store(key, LaunchShape{64 * bpc, 1});
        ctx.tuner->save();
    }
    solve_once(bpc);
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int l = 0; l < nlat; ++l) {
        const CgState &S = hs[l];
        lqs_cg_stats &o = stats[l];
        o.iters = S.iters;
        o.reliable_updates = S.nreliable;
        o.restarts = S.restarts;
        o.true_rel_residual = S.b2 > 0 ? std::sqrt(S.true_r2 / S.b2) : 0.0;
        o.seconds = secs;
        switch (S.phase) {
        case CG_CONVERGED: o.status = LQS_OK; break;
        case CG_BREAKDOWN: o.status = LQS_EBREAKDOWN; break;
        case CG_NONFINITE: o.status = LQS_ENONFINITE; break;
        default: o.status = LQS_ENOTCONV; break;
        }
    }
}

}  // namespace lqs
