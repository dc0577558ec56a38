// persistent.hip -- several independent even-odd CG solves (lattices of any
// size, each with its own links, mass and source) in ONE cooperative launch.
//
// Small lattices spend most of a multi-kernel CG iteration in launch gaps and
// global reductions (the latency the paper blames for the gap between its
// Dslash and CG numbers, Sec. 4.2).  Here the resident blocks are split into
// one group per lattice, sized in proportion to its sites; each group runs
// its own CG loop on its own lattice and synchronises only with itself (a
// one-block group needs no more than a block barrier), so the lattices
// advance independently.  One iteration has three phases separated by group
// barriers:
//   H: t = D_oe (r + beta p), the new search direction formed on the fly at
//      every neighbour read, rounded exactly as it will be stored
//   N: p = r + beta p (own site, stored), q = m^2 p - D_eo t, partials of <p,q>
//   U: alpha; x_lo += alpha p, r -= alpha q, partials of |r|^2
// then beta and the stop / reliable-update decisions, and, when asked for,
// the FP64 residual group (two more phases).  Every block of a group sums
// the group's tile partials itself in a fixed order, so all blocks of a
// group hold bit-identical scalars and take the same branches; partials are
// double-buffered so reading one reduction and writing the next need no
// barrier in between.  Group barriers wait with a bounded spin; a timeout
// raises a launch-wide abort flag that ends every group's loop.
#include <algorithm>
#include <chrono>
#include <cmath>

#include "hop.hpp"

namespace lqs {

static constexpr int PMAX_LAT = 256;

struct PLat {
    Geom g;
    LinkRef lo, hi;
    double m2;
    char *p, *q, *t, *r, *xlo, *t64;
    double *x;
    const double *b;
    int ntiles;         // tiles of this lattice (blockDim.x sites each)
    int block0;         // first block of this lattice's group
    int nblocks;        // blocks in the group
    double *part[2];    // tile partials, two buffers used alternately
};

struct GroupBar {
    uint32_t count;
    uint32_t gen;
};

// Barrier of the nb blocks of one group.  Each XCD has its own L2, so making
// a block's stores visible to blocks on other XCDs takes an agent-scope
// release (an L2 write-back) and reading theirs an agent-scope acquire (an L2
// invalidate); each block pays one of each per barrier: thread 0 releases,
// arrives with a relaxed atomic, spins with relaxed loads, then acquires.
// The last block to arrive resets the counter before it publishes the new
// generation with a release store.  A one-block group only needs the block
// barrier (its stores and loads go through the same compute unit).
__device__ __forceinline__ bool group_sync(GroupBar *gb, uint32_t *abort_flag, uint32_t nb, uint32_t &gen)
{
    __shared__ uint32_t aborted;
    if (nb == 1) {
        __syncthreads();
        return true;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const uint32_t old = __hip_atomic_fetch_add(&gb->count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (old == nb - 1) {
            __hip_atomic_store(&gb->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&gb->gen, gen + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            uint32_t spins = 0;
            while (__hip_atomic_load(&gb->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > (1u << 22)) {
                    __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                if ((spins & 255) == 0 && __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                    break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        gen += 1;
        aborted = __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    return aborted == 0;
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

template <int P, int R, int PA, int BS>
__global__ void __launch_bounds__(BS) persistent_cg_kernel(const PLat *lats, int nlat, CgState *st_out, GroupBar *bars,
                                                           uint32_t *abort_flag, int max_trips,
                                                           unsigned long long *clk)
{
    typedef typename RealOf<P>::type T;
    typedef typename RealOf<PA>::type TA;
    __shared__ CgState S;
    __shared__ PLat L;
    __shared__ int lat;
    if (threadIdx.x == 0) {
        int l = 0;
        while (l + 1 < nlat && (int)blockIdx.x >= lats[l + 1].block0) ++l;
        lat = l;
        L = lats[l];
        S = st_out[l];
    }
    __syncthreads();
    GroupBar *gb = bars + lat;
    const int nb = L.nblocks, lb = blockIdx.x - L.block0;
    // the group's device time: its first block's start and end (device wall clock)
    if (lb == 0 && threadIdx.x == 0) clk[2 * lat] = wall_clock64();
    uint32_t gen = 0;
    const int vh = L.g.vh;

    // new search direction at site cb: r + beta p, rounded as it will be stored
    auto direction = [&](TA beta, int cb) -> V3<T> {
        const V3<TA> rv = SpinorIO<PA>::load(L.r, vh, cb);
        const V3<TA> pv = vcast<TA>(SpinorIO<P>::load(L.p, vh, cb));
        V3<TA> o;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            o.c[a].re = fma(beta, pv.c[a].re, rv.c[a].re);
            o.c[a].im = fma(beta, pv.c[a].im, rv.c[a].im);
        }
        return Roundtrip<P>::apply(vcast<T>(o));
    };

    // ---- cold start: x = x_lo = 0, r = p = b, tile partials of |b|^2
    for (int tile = lb; tile < L.ntiles; tile += nb) {
        const int cb = tile * BS + threadIdx.x;
        double loc = 0.0;
        if (cb < vh) {
            const V3<double> bv = SpinorIO<F64>::load(L.b, vh, cb);
#pragma unroll
            for (int a = 0; a < 3; ++a) loc += bv.c[a].re * bv.c[a].re + bv.c[a].im * bv.c[a].im;
            SpinorIO<F64>::store(L.x, vh, cb, vzero<double>());
            SpinorIO<PA>::store(L.xlo, vh, cb, vzero<TA>());
            SpinorIO<PA>::store(L.r, vh, cb, vcast<TA>(bv));
            SpinorIO<P>::store(L.p, vh, cb, vcast<T>(bv));
        }
        const double s = block_sum(loc);
        if (threadIdx.x == 0) L.part[0][tile] = s;
    }
    bool aborted = !group_sync(gb, abort_flag, nb, gen);
    if (!aborted) {
        const double b2 = sum_partials(L.part[0], L.ntiles);
        if (threadIdx.x == 0) {
            S.b2 = b2;
            S.stop2 *= b2;
            S.rho = b2;
            S.max_rho = b2;
            S.true_r2 = b2;
            S.beta = 0.0;
            S.phase = (b2 == 0.0) ? CG_CONVERGED : (isfinite(b2) ? CG_RUNNING : CG_NONFINITE);
        }
        __syncthreads();
    }

    // FP64 residual of x + x_lo: t64 = D_oe (x + x_lo), then x += x_lo, x_lo = 0 and
    // r = b - (m^2 x - D_eo t64); returns |r|^2 (false when a barrier aborted).
    // store_r = false leaves r alone (measurement only).
    auto fp64_residual = [&](bool store_r, double &r2) -> bool {
        for (int tile = lb; tile < L.ntiles; tile += nb) {
            const int cb = tile * BS + threadIdx.x;
            if (cb >= vh) continue;
            const Site s = decode(L.g, cb, 1);
            const V3<double> acc = hop_site_fn<F64, 18>(L.g, L.hi, 1, s, cb, [&](int n) {
                V3<double> v = SpinorIO<F64>::load(L.x, vh, n);
                const V3<double> w = vcast<double>(SpinorIO<PA>::load(L.xlo, vh, n));
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    v.c[a].re += w.c[a].re;
                    v.c[a].im += w.c[a].im;
                }
                return v;
            });
            SpinorIO<F64>::store(L.t64, vh, cb, acc);
        }
        if (!group_sync(gb, abort_flag, nb, gen)) return false;
        for (int tile = lb; tile < L.ntiles; tile += nb) {
            const int cb = tile * BS + threadIdx.x;
            double loc = 0.0;
            if (cb < vh) {
                const Site s = decode(L.g, cb, 0);
                V3<double> acc;
                const bool act = true;
                hop_site<F64, 18, 1>(L.g, L.hi, 0, s, cb, L.t64, 0, &act, &acc);
                V3<double> xv = SpinorIO<F64>::load(L.x, vh, cb);
                const V3<double> lv = vcast<double>(SpinorIO<PA>::load(L.xlo, vh, cb));
                const V3<double> bv = SpinorIO<F64>::load(L.b, vh, cb);
                V3<double> rv;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    xv.c[a].re += lv.c[a].re;
                    xv.c[a].im += lv.c[a].im;
                    rv.c[a].re = bv.c[a].re - (L.m2 * xv.c[a].re - acc.c[a].re);
                    rv.c[a].im = bv.c[a].im - (L.m2 * xv.c[a].im - acc.c[a].im);
                    loc += rv.c[a].re * rv.c[a].re + rv.c[a].im * rv.c[a].im;
                }
                SpinorIO<F64>::store(L.x, vh, cb, xv);
                SpinorIO<PA>::store(L.xlo, vh, cb, vzero<TA>());
                if (store_r) SpinorIO<PA>::store(L.r, vh, cb, vcast<TA>(rv));
            }
            const double s = block_sum(loc);
            if (threadIdx.x == 0) L.part[0][tile] = s;
        }
        if (!group_sync(gb, abort_flag, nb, gen)) return false;
        r2 = sum_partials(L.part[0], L.ntiles);
        return true;
    };

    for (int trip = 0; !aborted && trip < max_trips && S.phase == CG_RUNNING; ++trip) {
        // ---- H: t = D_oe (r + beta p)
        {
            const TA beta = (TA)S.beta;
            for (int tile = lb; tile < L.ntiles; tile += nb) {
                const int cb = tile * BS + threadIdx.x;
                if (cb >= vh) continue;
                const Site s = decode(L.g, cb, 1);
                const V3<T> acc = hop_site_fn<P, R>(L.g, L.lo, 1, s, cb, [&](int n) { return direction(beta, n); });
                SpinorIO<P>::store(L.t, vh, cb, acc);
            }
        }
        if (!group_sync(gb, abort_flag, nb, gen)) {
            aborted = true;
            break;
        }

        // ---- N: p = r + beta p, q = m^2 p - D_eo t, tile partials of <p, q>
        for (int tile = lb; tile < L.ntiles; tile += nb) {
            const int cb = tile * BS + threadIdx.x;
            double dot = 0.0;
            if (cb < vh) {
                const V3<T> pv = direction((TA)S.beta, cb);
                const Site s = decode(L.g, cb, 0);
                V3<T> acc;
                const bool act = true;
                hop_site<P, R, 1>(L.g, L.lo, 0, s, cb, L.t, 0, &act, &acc);
                V3<T> qv;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    qv.c[a].re = (T)L.m2 * pv.c[a].re - acc.c[a].re;
                    qv.c[a].im = (T)L.m2 * pv.c[a].im - acc.c[a].im;
                    dot += (double)pv.c[a].re * (double)qv.c[a].re + (double)pv.c[a].im * (double)qv.c[a].im;
                }
                SpinorIO<P>::store(L.p, vh, cb, pv);
                SpinorIO<P>::store(L.q, vh, cb, qv);
            }
            const double s = block_sum(dot);
            if (threadIdx.x == 0) L.part[0][tile] = s;
        }
        if (!group_sync(gb, abort_flag, nb, gen)) {
            aborted = true;
            break;
        }
        {
            const double pq = sum_partials(L.part[0], L.ntiles);
            if (threadIdx.x == 0) {
                if (!isfinite(pq)) S.phase = CG_NONFINITE;
                else if (!(pq > 0.0)) S.phase = CG_BREAKDOWN;
                else S.alpha = S.rho / pq;
            }
            __syncthreads();
        }
        if (S.phase != CG_RUNNING) break;

        // ---- U: x_lo += alpha p, r -= alpha q, tile partials of |r|^2 (other buffer)
        {
            const TA alpha = (TA)S.alpha;
            for (int tile = lb; tile < L.ntiles; tile += nb) {
                const int cb = tile * BS + threadIdx.x;
                double loc = 0.0;
                if (cb < vh) {
                    const V3<TA> pv = vcast<TA>(SpinorIO<P>::load(L.p, vh, cb));
                    const V3<TA> qv = vcast<TA>(SpinorIO<P>::load(L.q, vh, cb));
                    V3<TA> xv = SpinorIO<PA>::load(L.xlo, vh, cb);
                    V3<TA> rv = SpinorIO<PA>::load(L.r, vh, cb);
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        xv.c[a].re += alpha * pv.c[a].re;
                        xv.c[a].im += alpha * pv.c[a].im;
                        rv.c[a].re -= alpha * qv.c[a].re;
                        rv.c[a].im -= alpha * qv.c[a].im;
                        loc += (double)rv.c[a].re * (double)rv.c[a].re + (double)rv.c[a].im * (double)rv.c[a].im;
                    }
                    SpinorIO<PA>::store(L.xlo, vh, cb, xv);
                    SpinorIO<PA>::store(L.r, vh, cb, rv);
                }
                const double s = block_sum(loc);
                if (threadIdx.x == 0) L.part[1][tile] = s;
            }
        }
        if (!group_sync(gb, abort_flag, nb, gen)) {
            aborted = true;
            break;
        }
        {
            const double r2 = sum_partials(L.part[1], L.ntiles);
            if (threadIdx.x == 0) p_fin_update(S, r2);
            __syncthreads();
        }
        if (!S.reliable_pending) continue;

        // ---- R: the FP64 residual (x += x_lo, x_lo = 0, r = b - M x)
        double r2 = 0.0;
        if (!fp64_residual(true, r2)) {
            aborted = true;
            break;
        }
        if (threadIdx.x == 0) p_fin_residual(S, r2);
        __syncthreads();
    }
    // A group that stopped without its final FP64 check (breakdown, non-finite
    // scalar, trip cap) still returns x = x + x_lo with its measured residual,
    // as the multi-kernel solver does.  After an aborted barrier x is undefined.
    if (!aborted && S.phase != CG_CONVERGED && S.phase != CG_MAXITER) {
        double r2 = 0.0;
        if (fp64_residual(false, r2) && threadIdx.x == 0) S.true_r2 = r2;
        __syncthreads();
    }
    if (lb == 0 && threadIdx.x == 0) {
        st_out[lat] = S;
        clk[2 * lat + 1] = wall_clock64();
    }
}

// ---------------------------------------------------------------------------

template <int P, int R, int PA> static const void *kernel_ptr(int bs)
{
    if (bs == 256) return (const void *)&persistent_cg_kernel<P, R, PA, 256>;
    if (bs == 512) return (const void *)&persistent_cg_kernel<P, R, PA, 512>;
    return (const void *)&persistent_cg_kernel<P, R, PA, 1024>;
}

static const void *pick_kernel(int prec, int recon, int bs)
{
    if (prec == F64) return recon == 12 ? kernel_ptr<F64, 12, F64>(bs) : kernel_ptr<F64, 18, F64>(bs);
    if (prec == F32) return recon == 12 ? kernel_ptr<F32, 12, F32>(bs) : kernel_ptr<F32, 18, F32>(bs);
    return recon == 12 ? kernel_ptr<F16, 12, F32>(bs) : kernel_ptr<F16, 18, F32>(bs);
}

// Blocks per lattice: proportional to its tiles, at least one, at most its
// tile count, summing to at most `total` (when total >= the lattice count).
static std::vector<int> split_blocks(const std::vector<int> &tiles, int total)
{
    const int n = (int)tiles.size();
    int64_t sum = 0;
    for (int t : tiles) sum += t;
    std::vector<int> nb(n);
    int used = 0;
    for (int l = 0; l < n; ++l) {
        const int want = (int)((int64_t)total * tiles[l] / (sum > 0 ? sum : 1));
        nb[l] = std::max(1, std::min(want, tiles[l]));
        used += nb[l];
    }
    std::vector<int> order(n);
    for (int l = 0; l < n; ++l) order[l] = l;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return tiles[a] > tiles[b]; });
    for (int l : order)
        while (used < total && nb[l] < tiles[l]) {
            ++nb[l];
            ++used;
        }
    for (int l : order)
        while (used > total && nb[l] > 1) {
            --nb[l];
            --used;
        }
    return nb;
}

void persistent_solve(Ctx &ctx, const std::vector<PersistentProblem> &probs, const lqs_cg_params &prm,
                      lqs_cg_stats *stats, hipStream_t s)
{
    auto t0 = std::chrono::steady_clock::now();
    const int nlat = (int)probs.size();
    LQS_REQUIRE(nlat >= 1 && nlat <= PMAX_LAT, LQS_EUNSUPPORTED, "persistent solve takes 1..256 lattices");
    LQS_REQUIRE(!prm.use_x0, LQS_EUNSUPPORTED, "persistent solve starts from x = 0");
    int coop = 0;
    LQS_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, ctx.device));
    LQS_REQUIRE(coop, LQS_EUNSUPPORTED, "device has no cooperative launch");
    const int prec = prm.inner_prec, recon = prm.inner_recon == 12 ? 12 : 18;
    const int pa = prec == F64 ? F64 : F32;
    const bool mixed = prec != F64;

    // fields and descriptors (partials sized for the smallest tile)
    std::vector<PLat> L(nlat);
    size_t part_total = 0;
    for (int l = 0; l < nlat; ++l) part_total += (size_t)((probs[l].gauge->vh + 255) / 256);
    double *partials = (double *)ctx.workspace("pcg.partials", 2 * sizeof(double) * part_total);
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
    }
    PLat *dL = (PLat *)ctx.workspace("pcg.desc", sizeof(PLat) * nlat);
    CgState *dS = (CgState *)ctx.workspace("pcg.state", sizeof(CgState) * nlat);
    // one group barrier per lattice, then the abort word
    const size_t bar_bytes = sizeof(GroupBar) * PMAX_LAT + 16;
    GroupBar *bars = (GroupBar *)ctx.workspace("pcg.bar", bar_bytes);
    uint32_t *abort_flag = (uint32_t *)(bars + PMAX_LAT);
    unsigned long long *clk = (unsigned long long *)ctx.workspace("pcg.clk", 2 * sizeof(unsigned long long) * nlat);
    std::vector<unsigned long long> hclk(2 * nlat);
    int clk_khz = 0;
    LQS_HIP(hipDeviceGetAttribute(&clk_khz, hipDeviceAttributeWallClockRate, ctx.device));
    std::vector<CgState> init(nlat), hs(nlat);
    const int rel_interval = mixed ? (prm.reliable_interval > 0 ? prm.reliable_interval : 100) : 0;
    const double delta =
        mixed ? (prm.reliable_delta > 0 ? prm.reliable_delta : default_reliable_delta(prm.inner_prec)) : 0.0;
    for (auto &S : init) {
        S = CgState{};
        S.stop2 = prm.tol * prm.tol;
        S.delta2 = delta * delta;
        S.rel_interval = rel_interval;
        S.max_iter = prm.max_iter;
        S.phase = CG_RUNNING;
    }
    const int max_trips = prm.max_iter + 8;
    uint32_t habort = 0;

    // One complete solve with tiles of `bs` sites and `bpc` resident blocks per CU.
    auto solve_once = [&](int bs, int bpc) {
        const void *fn = pick_kernel(prec, recon, bs);
        int per_cu = 0;
        LQS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, bs, 0));
        LQS_REQUIRE(per_cu >= 1, LQS_EUNSUPPORTED, "persistent kernel does not fit on a compute unit");
        std::vector<int> tiles(nlat);
        int total_tiles = 0;
        for (int l = 0; l < nlat; ++l) {
            tiles[l] = (int)((probs[l].gauge->vh + bs - 1) / bs);
            total_tiles += tiles[l];
        }
        const int resident = std::min(bpc, per_cu) * ctx.num_cu;
        const std::vector<int> nb = split_blocks(tiles, std::max(nlat, std::min(resident, total_tiles)));
        size_t off = 0;
        int b0 = 0;
        for (int l = 0; l < nlat; ++l) {
            L[l].ntiles = tiles[l];
            L[l].block0 = b0;
            L[l].nblocks = nb[l];
            b0 += nb[l];
            L[l].part[0] = partials + off;
            L[l].part[1] = partials + part_total + off;
            off += tiles[l];
        }
        LQS_REQUIRE(b0 <= resident, LQS_EUNSUPPORTED, "more lattices than resident blocks");
        LQS_HIP(hipMemcpyAsync(dL, L.data(), sizeof(PLat) * nlat, hipMemcpyHostToDevice, s));
        LQS_HIP(hipMemcpyAsync(dS, init.data(), sizeof(CgState) * nlat, hipMemcpyHostToDevice, s));
        LQS_HIP(hipMemsetAsync(bars, 0, bar_bytes, s));
        int n = nlat;
        int trips = max_trips;
        void *args[] = {(void *)&dL, (void *)&n,    (void *)&dS,   (void *)&bars,
                        (void *)&abort_flag, (void *)&trips, (void *)&clk};
        LQS_HIP(hipLaunchCooperativeKernel(fn, dim3(b0), dim3(bs), args, 0, s));
        // From here the kernel and the copies into host memory may be in flight:
        // on any error the stream is drained before the host buffers go away.
        try {
            LQS_HIP(hipMemcpyAsync(hs.data(), dS, sizeof(CgState) * nlat, hipMemcpyDeviceToHost, s));
            LQS_HIP(hipMemcpyAsync(&habort, abort_flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
            LQS_HIP(hipMemcpyAsync(hclk.data(), clk, 2 * sizeof(unsigned long long) * nlat, hipMemcpyDeviceToHost,
                                   s));
            LQS_HIP(hipStreamSynchronize(s));
        } catch (...) {
            (void)hipStreamSynchronize(s);
            throw;
        }
        LQS_REQUIRE(habort == 0, LQS_EHIP, "persistent solve: group barrier timed out");
    };

    // Tuned: threads per block (= sites per tile) and resident blocks per CU,
    // stored as LaunchShape{block, rhs_per_thread = blocks per CU}; the key
    // names every lattice of the batch.
    std::string key = std::string(ctx.prop.gcnArchName) + "|persistent|p" + std::to_string(prec) + "|r" +
                      std::to_string(recon);
    for (const PLat &d : L)
        key += "|" + std::to_string(d.g.n[0]) + "x" + std::to_string(d.g.n[1]) + "x" + std::to_string(d.g.n[2]) +
               "x" + std::to_string(d.g.n[3]);
    LaunchShape best{1024, 1};  // the shape the search picks on the uneven 16^4 / 24^3x8 / 32^3x8 batch
    LaunchShape t;
    if (ctx.tuner && ctx.tuner->lookup(key, t, 1024)) {
        best = t;
    } else if (ctx.tuning && ctx.tuner) {
        double best_s = 1e30;
        const LaunchShape cands[] = {{256, 4}, {256, 2}, {256, 1}, {512, 2}, {512, 1}, {1024, 1}};
        for (const LaunchShape &c : cands) {
            auto a0 = std::chrono::steady_clock::now();
            solve_once(c.block, c.rhs_per_thread);
            const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - a0).count();
            if (dt < best_s) {
                best_s = dt;
                best = c;
            }
        }
        ctx.tuner->store(key, best);
        ctx.tuner->save();
    }
    solve_once(best.block, best.rhs_per_thread);
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int l = 0; l < nlat; ++l) {
        const CgState &S = hs[l];
        lqs_cg_stats &o = stats[l];
        o.iters = S.iters;
        o.reliable_updates = S.nreliable;
        o.restarts = S.restarts;
        o.true_rel_residual = S.b2 > 0 ? std::sqrt(S.true_r2 / S.b2) : 0.0;
        o.seconds = secs;
        o.device_seconds = clk_khz > 0 ? (double)(hclk[2 * l + 1] - hclk[2 * l]) / (1e3 * clk_khz) : 0.0;
        cg_fill_rates(o, *probs[l].gauge, prec, recon, 1);
        switch (S.phase) {
        case CG_CONVERGED: o.status = LQS_OK; break;
        case CG_BREAKDOWN: o.status = LQS_EBREAKDOWN; break;
        case CG_NONFINITE: o.status = LQS_ENONFINITE; break;
        default: o.status = LQS_ENOTCONV; break;
        }
    }
}

}  // namespace lqs
