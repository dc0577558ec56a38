// dslash.hip -- the staggered hop D_{p,1-p} (eq. (1), Sec. 4.2) and its
// adjoint, for one or several right-hand sides (Sec. 4.3, "NMULTI").
//
// One thread computes one output site for K right-hand sides: it streams the
// four forward links of its own parity and the four backward links of the
// other parity once (coalesced word-major arrays), and gathers the eight
// neighbouring colour vectors, which nearby threads share through the caches.
// The stencil is bound by HBM bandwidth (570 flop per site against 1584 bytes
// in FP64), so there is no matrix-core path.
#include "hop.hpp"

namespace lqs {


template <int P, int R, int K, bool DAG, int LF>
__global__ void __launch_bounds__(512) hop_kernel(Geom g, LinkRef L, int parity, int nrhs, const char *in,
                                                  int64_t in_stride, char *out, int64_t out_stride,
                                                  const CgState *gate, int gate_mode, int ngroups, TileMap tmap)
{
    typedef typename RealOf<P>::type T;
    int grp;
    const int tile = tile_group(ngroups, tmap, g.n[3], grp);
    const int c0 = tile * blockDim.x;
    if (tile < 0 || c0 >= g.vh) return;  // padding tile (whole block)
    const int cb = c0 + threadIdx.x;
    const int r0 = grp * K;
    bool active[K];
    bool any = false;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        active[j] = (r0 + j < nrhs) && gate_open(gate, gate_mode, r0 + j);
        any |= active[j];
    }
    if (!any) return;  // uniform over the block
    extern __shared__ __align__(16) char win[];
    int w0 = 0, wlen = 0;
    const int wstride = lds_window_stride(g, P);
    if (LF & LF_LDS) stage_block_window<P, K>(g, c0, in + r0 * in_stride, in_stride, active, win, wstride, w0, wlen);
    if (cb >= g.vh) return;
    const Site s = decode(g, cb, parity);
    V3<T> acc[K];
    hop_site<P, R, K, LF>(g, L, parity, s, cb, in + r0 * in_stride, in_stride, active, acc, win, wstride, w0, wlen);
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (!active[j]) continue;
        V3<T> o = acc[j];
        if (DAG) {
#pragma unroll
            for (int a = 0; a < 3; ++a) o.c[a] = {-o.c[a].re, -o.c[a].im};
        }
        SpinorIO<P>::store(out + (r0 + j) * out_stride, g.vh, cb, o);
    }
}

template <int P, int R, int K>
static void launch_k(const Geom &g, LinkRef L, int dagger, int parity, int nrhs, const void *in, void *out,
                     const CgState *gate, int gate_mode, LaunchShape sh, hipStream_t s)
{
    const int64_t stride = field_bytes(g, P, 1);
    const int G = (nrhs + K - 1) / K;
    const TileMap tmap = tile_map(g, sh.block, sh.xcd_slab, time_run(g, sh.block, nrhs, P, sh.trun));
    const dim3 grid(tile_map_blocks(g, sh.block, tmap, G));
    const size_t lds = hop_lds_bytes(g, P, K, sh);
    const int lf = (L.temporal ? LF_TEMPORAL : 0) | (sh.stream_links ? LF_STREAM : 0) | (lds ? LF_LDS : 0);
#define LQS_HOP(DAG, LF)                                                                                         \
    hipLaunchKernelGGL((hop_kernel<P, R, K, DAG, LF>), grid, dim3(sh.block), lds, s, g, L, parity, nrhs,          \
                       (const char *)in, stride, (char *)out, stride, gate, gate_mode, G, tmap)
#define LQS_HOP_LF(LF)                                                                                           \
    if (dagger) LQS_HOP(true, LF);                                                                                \
    else LQS_HOP(false, LF)
    if (sh.prefetch && !lds) {
        switch (lf) {
        case 0: LQS_HOP_LF(LF_PREFETCH); break;
        case LF_TEMPORAL: LQS_HOP_LF(LF_PREFETCH | LF_TEMPORAL); break;
        case LF_STREAM: LQS_HOP_LF(LF_PREFETCH | LF_STREAM); break;
        default: LQS_HOP_LF(LF_PREFETCH | LF_TEMPORAL | LF_STREAM); break;
        }
        LQS_HIP(hipGetLastError());
        return;
    }
    switch (lf) {
    case 0: LQS_HOP_LF(0); break;
    case LF_TEMPORAL: LQS_HOP_LF(LF_TEMPORAL); break;
    case LF_STREAM: LQS_HOP_LF(LF_STREAM); break;
    case LF_TEMPORAL | LF_STREAM: LQS_HOP_LF(LF_TEMPORAL | LF_STREAM); break;
    case LF_LDS: LQS_HOP_LF(LF_LDS); break;
    case LF_LDS | LF_STREAM: LQS_HOP_LF(LF_LDS | LF_STREAM); break;
    case LF_LDS | LF_TEMPORAL: LQS_HOP_LF(LF_LDS | LF_TEMPORAL); break;
    default: LQS_HOP_LF(LF_LDS | LF_TEMPORAL | LF_STREAM); break;
    }
#undef LQS_HOP_LF
#undef LQS_HOP
    LQS_HIP(hipGetLastError());
}

template <int P, int R>
static void launch_pr(const Geom &g, LinkRef L, int dagger, int parity, int nrhs, const void *in, void *out,
                      const CgState *gate, int gate_mode, LaunchShape sh, hipStream_t s)
{
    switch (sh.rhs_per_thread) {
    case 1: launch_k<P, R, 1>(g, L, dagger, parity, nrhs, in, out, gate, gate_mode, sh, s); break;
    case 2: launch_k<P, R, 2>(g, L, dagger, parity, nrhs, in, out, gate, gate_mode, sh, s); break;
    case 4: launch_k<P, R, 4>(g, L, dagger, parity, nrhs, in, out, gate, gate_mode, sh, s); break;
    default: throw Error(LQS_EINVAL, "rhs_per_thread must be 1, 2 or 4");
    }
}

void launch_hop_gated(const Geom &g, LinkRef L, int prec, int recon, int dagger, int parity, int nrhs,
                      const void *in, void *out, const CgState *gate, int gate_mode, LaunchShape sh, hipStream_t s)
{
    if (prec == F64 && recon == 18) launch_pr<F64, 18>(g, L, dagger, parity, nrhs, in, out, gate, gate_mode, sh, s);
    else if (prec == F64) launch_pr<F64, 12>(g, L, dagger, parity, nrhs, in, out, gate, gate_mode, sh, s);
    else if (prec == F32 && recon == 18) launch_pr<F32, 18>(g, L, dagger, parity, nrhs, in, out, gate, gate_mode, sh, s);
    else if (prec == F32) launch_pr<F32, 12>(g, L, dagger, parity, nrhs, in, out, gate, gate_mode, sh, s);
    else if (recon == 18) launch_pr<F16, 18>(g, L, dagger, parity, nrhs, in, out, gate, gate_mode, sh, s);
    else launch_pr<F16, 12>(g, L, dagger, parity, nrhs, in, out, gate, gate_mode, sh, s);
}

// Default shapes from measured sweeps on 32^4, 32^3x8 and 64^3x16: from 4
// vectors on, 4 right-hand sides per thread in 256-thread blocks with the
// pencil block -> tile map in runs of time slices (time_run) and prefetched
// words (steady state, 64^3x16, 4 vectors: FP16 12-real 154 against 197 us
// without prefetch, FP32 250 against 331, FP64 12-real 501 against 623; 16
// vectors 10-20 % faster on 32^4 and 64^3x16; the pencil map against
// time-inner over all slices: 32^4 FP16 12-real 4 vectors 33.7 against
// 41.9 us, FP64 18-real 16 vectors 458 against 499, 64^3x16 FP64 18-real
// 16 vectors 1739 against 1946, 32^3x8 FP32 12-real 16 vectors 38 against
// 49, elsewhere within 3 %); 2 per thread in 128-thread blocks for 2-3 vectors, also
// prefetched (3 vectors at 64^3x16: FP32 12-real 252 against 336 us, FP64
// 18-real 688 against 903 us; 2 vectors 0-8 % faster).  Links are streamed
// when their footprint exceeds STREAM_LINK_BYTES and one group of right-hand
// sides covers all of them; with several groups the blocks of one site tile
// reuse the links from L2 (see tile_group) and cached loads win.  One vector
// on a lattice of at most PREFETCH_MAX_SITES sites per parity (a few waves per
// SIMD) is prefetched too; on larger ones prefetch is within -7 .. +5 % and
// left to the tuner.
static constexpr int64_t PREFETCH_MAX_SITES = (int64_t)1 << 18;
LaunchShape default_hop_shape(const LinkRef &L, int nrhs)
{
    LaunchShape sh;
    if (nrhs >= 4) {
        sh.block = 256;
        sh.rhs_per_thread = 4;
        sh.xcd_slab = 3;
        sh.prefetch = 1;
    } else if (nrhs >= 2) {
        sh.block = 128;
        sh.rhs_per_thread = 2;
        sh.prefetch = 1;
    } else {
        sh.block = 256;
        sh.rhs_per_thread = 1;
    }
    sh.stream_links = (8 * L.block_bytes >= STREAM_LINK_BYTES && nrhs <= sh.rhs_per_thread) ? 1 : 0;
    if (sh.rhs_per_thread == 1) sh.prefetch = L.pitch <= PREFETCH_MAX_SITES ? 1 : 0;
    return sh;
}

void launch_hop_shape(const Geom &g, LinkRef links, int prec, int recon, int dagger, int out_parity, int nrhs,
                      const void *in, void *out, const CgState *gate, LaunchShape shape, hipStream_t s)
{
    launch_hop_gated(g, links, prec, recon, dagger, out_parity, nrhs, in, out, gate, gate ? 1 : 0, shape, s);
}

// ---------------------------------------------------------------------------
// profiling of hop launches with HIP events on the launch stream

void prof_begin(Ctx &ctx, hipStream_t s)
{
    if (!ctx.profiling) return;
    if (ctx.prof_used == ctx.prof_events.size()) {
        hipEvent_t a, b;
        LQS_HIP(hipEventCreate(&a));
        LQS_HIP(hipEventCreate(&b));
        ctx.prof_events.push_back({a, b});
        ctx.prof_keys.push_back({0, 0});
        ctx.prof_sites.push_back(0);
    }
    LQS_HIP(hipEventRecord(ctx.prof_events[ctx.prof_used].first, s));
}

void prof_end(Ctx &ctx, int prec, int recon, int64_t sites, hipStream_t s)
{
    if (!ctx.profiling) return;
    LQS_HIP(hipEventRecord(ctx.prof_events[ctx.prof_used].second, s));
    ctx.prof_keys[ctx.prof_used] = {prec, recon == 12 ? 1 : 0};
    ctx.prof_sites[ctx.prof_used] = sites;
    ++ctx.prof_used;
}

void launch_hop(Ctx &ctx, const Gauge &gauge, int prec, int recon, int dagger, int out_parity, int nrhs,
                const void *in, void *out, hipStream_t s, const CgState *gate)
{
    const LinkRef L = gauge.ref(prec, recon);
    LaunchShape sh = default_hop_shape(L, nrhs);
    if (ctx.tuner) ctx.tuner->lookup(tune_key(ctx, gauge.temporal ? "hop_tg" : "hop", gauge.g, prec, recon, nrhs), sh);
    prof_begin(ctx, s);
    launch_hop_gated(gauge.g, L, prec, recon, dagger, out_parity, nrhs, in, out, gate, gate ? 1 : 0, sh, s);
    prof_end(ctx, prec, recon, (int64_t)gauge.vh * nrhs, s);
}

}  // namespace lqs
