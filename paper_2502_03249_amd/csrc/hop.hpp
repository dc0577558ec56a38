// hop.hpp -- eq. (1) of the paper evaluated at one output site for K
// right-hand sides that share the links (Sec. 4.2 for the operator, Sec. 4.3
// for applying it to several vectors with one read of each link).
#pragma once
#include "dev.hpp"
#include "lqs_impl.hpp"

namespace lqs {

// acc[j] = sum_mu [eps_mu(x) U_{x,mu} in_j(x+mu) - eps_mu(x-mu) U^dag_{x-mu,mu} in_j(x-mu)]
// for the site cb of parity `parity` (decoded into s).  LF holds link flags:
// LF_TEMPORAL, the links are in temporal gauge (U_t = 1 off the last time
// slice) and those t-links are not read from the link arrays (without it every
// link is read, also correct for temporal-gauge links, just slower);
// LF_STREAM, link words are fetched with streaming loads; LF_PREFETCH (no
// LDS window), the memory words of a group of directions are all requested
// before any is used.  Inactive right-hand sides are skipped and keep
// acc = 0.  `in` points at right-hand side 0 of the input field (parity
// 1 - parity); consecutive sides are in_stride bytes apart.
enum { LF_TEMPORAL = 1, LF_STREAM = 2, LF_LDS = 4, LF_PREFETCH = 8 };

// Block -> (site tile, right-hand-side group).  Consecutive block indices go
// to the 8 XCDs in turn, each with its own L2; four maps build on that
// (TileMap, from tile_map below):
//  - round robin (TM_RR): tile t runs on XCD t mod 8, and the G blocks of one
//    tile are 8 block indices apart, so they run on the same XCD in close
//    succession and the links they share come from HBM once, then from that
//    XCD's L2.  Neighbour tiles a multiple of 8 tiles away share the XCD.
//  - slab (TM_SLAB, n tiles per XCD): XCD x sweeps the contiguous tiles
//    [x n, (x + 1) n), so every neighbour except those across the slab ends
//    is in its L2.
//  - time-inner (TM_TIME, n = S tiles per time slice): the tiles s of a time
//    slice go to XCD s mod 8, and each XCD runs `run` consecutive time slices
//    of one of its tiles before its next tile, then the next run of slices.
//    The t neighbours of a tile were read one tile earlier and the z
//    neighbours `run` tiles earlier, on the same XCD; the lexicographic sweep
//    instead reads a t neighbour a whole time slice later, which with several
//    right-hand sides no longer fits in L2.
//  - pencil (TM_PENCIL, also per runs of time slices): within a time slice the
//    tiles are ordered band by band (a band: the tiles at one position in
//    their z plane, p tiles per plane) with z inner, and XCD x takes the x-th
//    eighth of that order.  Its z neighbours then stay on the XCD also when a
//    plane holds fewer than 8 tiles, where time-inner spreads them over XCDs.
// Shorter runs bound what an XCD reads between a tile and its z neighbour
// (run tiles for all right-hand sides) at the cost of re-reading the input
// slices at the run ends.  Returns the tile, or -1 for a padding block.
// Grids: tile_map_blocks.
enum { TM_RR = 0, TM_SLAB = 1, TM_TIME = 2, TM_PENCIL = 3 };
struct TileMap {
    int kind = TM_RR;
    int n = 0;    // TM_SLAB: tiles per XCD; TM_TIME, TM_PENCIL: tiles per time slice
    int p = 1;    // TM_PENCIL: tiles per z plane
    int run = 1;  // TM_TIME, TM_PENCIL: time slices per run (the last run may be shorter)
};
__host__ __device__ __forceinline__ int tile_of_block(int b, int G, const TileMap &m, int nt, int &grp)
{
    const int xcd = b & 7, q = b >> 3;
    grp = q % G;
    const int qq = q / G;
    if (m.kind == TM_RR) return qq * 8 + xcd;
    if (m.kind == TM_SLAB) return xcd * m.n + qq;
    const int S = m.n, per = (S + 7) >> 3;  // tiles of one slice per XCD
    const int rb = qq / (per * m.run), r = qq - rb * per * m.run;
    const int len = m.run < nt - rb * m.run ? m.run : nt - rb * m.run;
    const int k = r / len, t = rb * m.run + (r - k * len);
    int s;
    if (m.kind == TM_TIME) {
        s = k * 8 + xcd;
    } else {
        const int o = xcd * per + k, nz = S / m.p;
        s = o < S ? (o % nz) * m.p + o / nz : S;
    }
    return s < S ? t * S + s : -1;
}
__device__ __forceinline__ int tile_group(int G, const TileMap &m, int nt, int &grp)
{
    return tile_of_block(blockIdx.x, G, m, nt, grp);
}

// The round-robin map keeps the z and t neighbours of a tile on its XCD when
// the z stride (Nx Ny / 2 sites) is a whole number of 8-tile strides; the
// slab map is used otherwise (mode -1).  Modes 0, 1, 2, 3 ask for round
// robin, slab, time-inner and pencil; time-inner needs whole tiles per time
// slice and pencil whole tiles per z plane (else time-inner), and they fall
// back to the automatic choice otherwise.  `run` (0: all Nt) is their run of
// time slices.
inline bool xcd_slab_auto(const Geom &g, int block) { return ((int64_t)g.n[0] * g.n[1] / 2) % (8 * block) != 0; }
inline TileMap tile_map(const Geom &g, int block, int mode, int run = 0)
{
    TileMap m;
    const int tiles = (g.vh + block - 1) / block;
    const int64_t slice = (int64_t)g.vh / g.n[3], plane = (int64_t)g.n[0] * g.n[1] / 2;
    const int nrun = run > 0 && run < g.n[3] ? run : g.n[3];
    if (mode == 2 && slice % block == 0) {
        m.kind = TM_TIME;
        m.n = (int)(slice / block);
        m.run = nrun;
        return m;
    }
    if (mode == 3 && plane % block == 0) {
        m.kind = TM_PENCIL;
        m.n = (int)(slice / block);
        m.p = (int)(plane / block);
        m.run = nrun;
        return m;
    }
    if (mode == 3 && slice % block == 0) {
        m.kind = TM_TIME;
        m.n = (int)(slice / block);
        m.run = nrun;
        return m;
    }
    const bool slab = (mode >= 2 || mode < 0) ? xcd_slab_auto(g, block) : mode != 0;
    if (slab) {
        m.kind = TM_SLAB;
        m.n = (tiles + 7) / 8;
    }
    return m;
}
// Automatic run of time slices (LaunchShape::trun < 0): all of them up to 8
// slices; on longer lattices the longest run of at most 8 (down to 2) for
// which the input colour vectors an XCD reads between a tile and its z
// neighbour, 2 run tiles of `block` sites and all right-hand sides, stay
// within 2 MiB of its 4 MiB L2.  Measured FP64 18-real, 16 vectors: 64^3x16
// 1739 us at runs of 4 against 1959 over all 16 slices; 32^4 442 against 567.
inline int time_run(const Geom &g, int block, int nrhs, int prec, int trun)
{
    if (trun >= 0) return trun;
    if (g.n[3] <= 8) return 0;
    int r = 8;
    while (r > 2 && 2ll * r * block * nrhs * spinor_bytes_per_site(prec) > (2ll << 20)) r /= 2;
    return r;
}
inline unsigned tile_map_blocks(const Geom &g, int block, const TileMap &m, int G)
{
    const int tiles = (g.vh + block - 1) / block;
    if (m.kind == TM_RR && G == 1) return tiles;
    if (m.kind == TM_RR || m.kind == TM_SLAB) return ((tiles + 7) / 8) * 8 * G;
    return ((m.n + 7) / 8) * 8 * g.n[3] * G;
}

// Gates of the CG kernels on the state of one right-hand side.  0: always;
// 1: while RUNNING; 2: an FP64 residual update is pending; 3: pending while
// RUNNING (a periodic reliable update); 4: pending after the iterated
// residual met the target (the update that decides convergence).
__device__ __forceinline__ bool gate_state(const CgState &S, int gate_mode)
{
    switch (gate_mode) {
    case 0: return true;
    case 1: return S.phase == CG_RUNNING;
    case 2: return S.reliable_pending != 0;
    case 3: return S.reliable_pending != 0 && S.phase == CG_RUNNING;
    default: return S.reliable_pending != 0 && S.phase != CG_RUNNING;
    }
}
__device__ __forceinline__ bool gate_open(const CgState *gate, int gate_mode, int r)
{
    return gate_mode == 0 || gate_state(gate[r], gate_mode);
}

// LDS bytes of the staged input window of a hop launch: K sides of B + Nx + 2
// sites; 0 (no staging) unless the shape asks for it and the window fits in
// 64 KiB.
inline size_t hop_lds_bytes(const Geom &g, int prec, int K, const LaunchShape &sh)
{
    if (!sh.lds) return 0;
    const size_t b = (size_t)K * spinor_bytes_per_site(prec) * (sh.block + g.n[0] + 2);
    return b <= 65536 ? b : 0;
}

// Copy sites [w0, w0 + wlen) of one colour-vector field into an LDS window
// laid out like the field with wlen sites per plane.
template <int P> __device__ __forceinline__ void stage_window(const char *src, int64_t vh, char *dst, int w0, int wlen);
template <> __device__ __forceinline__ void stage_window<F64>(const char *src, int64_t vh, char *dst, int w0, int wlen)
{
    for (int k = 0; k < 3; ++k)
        for (int i = threadIdx.x; i < wlen; i += blockDim.x)
            ((double2 *)dst)[k * wlen + i] = ((const double2 *)src)[k * vh + w0 + i];
}
template <> __device__ __forceinline__ void stage_window<F32>(const char *src, int64_t vh, char *dst, int w0, int wlen)
{
    for (int i = threadIdx.x; i < wlen; i += blockDim.x) {
        ((float4 *)dst)[i] = ((const float4 *)src)[w0 + i];
        ((float2 *)((float4 *)dst + wlen))[i] = ((const float2 *)((const float4 *)src + vh))[w0 + i];
    }
}
template <> __device__ __forceinline__ void stage_window<F16>(const char *src, int64_t vh, char *dst, int w0, int wlen)
{
    (void)vh;
    for (int i = threadIdx.x; i < wlen; i += blockDim.x) ((uint4 *)dst)[i] = ((const uint4 *)src)[w0 + i];
}

// LF_LDS staging for the block whose sites start at c0: the x and y neighbours
// of [c0, c0 + B) lie in [c0 - Nx/2 - 1, c0 + B + Nx/2 + 1) except across
// periodic boundaries (read from memory).  Copies that window of every side j
// with stage[j] set (block-uniform) into win + j * wstride and waits for the
// block; returns the window as [w0, w0 + wlen).
__device__ __forceinline__ int lds_window_stride(const Geom &g, int prec)
{
    return (int)(spinor_bytes_per_site(prec) * (blockDim.x + g.n[0] + 2));
}
template <int P, int K>
__device__ __forceinline__ void stage_block_window(const Geom &g, int c0, const char *in, int64_t in_stride,
                                                   const bool *stage, char *win, int wstride, int &w0, int &wlen)
{
    const int h = g.n[0] / 2 + 1;
    w0 = c0 - h > 0 ? c0 - h : 0;
    const int w1 = c0 + (int)blockDim.x + h < g.vh ? c0 + (int)blockDim.x + h : g.vh;
    wlen = w1 - w0;
#pragma unroll
    for (int j = 0; j < K; ++j)
        if (stage[j]) stage_window<P>(in + j * in_stride, g.vh, win + j * wstride, w0, wlen);
    __syncthreads();
}

// hop_site for FP16 storage: the products run on the stored binary16 words
// (accum_h) instead of decoded binary32 values, which takes about half the
// vector instructions; the loads, their order and grouping (LF_PREFETCH) and
// the LDS window are those of hop_site below, and every variant sums in the
// same order, so they agree bit for bit.
template <int R, int K, int LF>
__device__ __forceinline__ void hop_site_h(const Geom &g, const LinkRef &L, int parity, const Site &s, int cb,
                                           const char *in, int64_t in_stride, const bool *active, V3<float> *acc,
                                           const char *win, int win_stride, int w0, int wlen)
{
    constexpr bool TG = (LF & LF_TEMPORAL) != 0, NT = (LF & LF_STREAM) != 0;
    typedef LinkIO<F16, R, NT> LIO;
    typedef SpinorIO<F16> SIO;
    const char *lb = (const char *)L.base;
#pragma unroll
    for (int j = 0; j < K; ++j) acc[j] = vzero<float>();
    if constexpr ((LF & LF_PREFETCH) != 0) {
        static_assert((LF & LF_LDS) == 0, "prefetch: no LDS window");
        constexpr int GRP = K == 1 ? 8 : K == 2 ? 4 : 2;
#pragma unroll
        for (int d0 = 0; d0 < 8; d0 += GRP) {
            typename LIO::Raw lr[GRP];
            W16 vr[GRP][K];
#pragma unroll
            for (int k = 0; k < GRP; ++k) {
                const int d = d0 + k, mu = d >> 1;
                const bool fwd = (d & 1) == 0;
                const bool unit = TG && mu == 3 && (s.tunit & (fwd ? 1u : 2u));
                const int at = unit ? g.vh : (fwd ? cb : s.bwd[mu]);
                lr[k] = LIO::load_raw(lb + (2 * mu + (fwd ? parity : 1 - parity)) * L.block_bytes, L.pitch, at);
#pragma unroll
                for (int j = 0; j < K; ++j)
                    vr[k][j] = SIO::load_raw(in + (active[j] ? j : 0) * in_stride, g.vh, fwd ? s.fwd[mu] : s.bwd[mu]);
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int k = 0; k < GRP; ++k) {
                const int d = d0 + k, mu = d >> 1;
                const M3H u = link_words<R>(lr[k]);
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    if (!active[j]) continue;
                    if ((d & 1) == 0) accum_h<true, R>(acc[j], u, vr[k][j], (s.negf >> mu) & 1);
                    else accum_h<false, R>(acc[j], u, vr[k][j], !((s.negb >> mu) & 1));
                }
            }
        }
        return;
    }
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const bool nf = (s.negf >> mu) & 1;
        const bool nb = !((s.negb >> mu) & 1);
        const bool uf_unit = TG && mu == 3 && (s.tunit & 1u);
        const bool ub_unit = TG && mu == 3 && (s.tunit & 2u);
        const M3H uf = link_words<R>(LIO::load_raw(lb + (2 * mu + parity) * L.block_bytes, L.pitch, uf_unit ? g.vh : cb));
#pragma unroll
        for (int j = 0; j < K; ++j) {
            if (!active[j]) continue;
            const int nbr = s.fwd[mu];
            const bool lw = (LF & LF_LDS) && mu < 2 && nbr >= w0 && nbr < w0 + wlen;
            const W16 v = lw ? SIO::load_raw(win + j * win_stride, wlen, nbr - w0) : SIO::load_raw(in + j * in_stride, g.vh, nbr);
            accum_h<true, R>(acc[j], uf, v, nf);
        }
        const M3H ub =
            link_words<R>(LIO::load_raw(lb + (2 * mu + 1 - parity) * L.block_bytes, L.pitch, ub_unit ? g.vh : s.bwd[mu]));
#pragma unroll
        for (int j = 0; j < K; ++j) {
            if (!active[j]) continue;
            const int nbr = s.bwd[mu];
            const bool lw = (LF & LF_LDS) && mu < 2 && nbr >= w0 && nbr < w0 + wlen;
            const W16 v = lw ? SIO::load_raw(win + j * win_stride, wlen, nbr - w0) : SIO::load_raw(in + j * in_stride, g.vh, nbr);
            accum_h<false, R>(acc[j], ub, v, nb);
        }
    }
}

// LF_LDS: the x and y neighbours of a block's sites come from an LDS window
// (win: right-hand side 0; win_stride bytes per side; sites [w0, w0 + wlen)).
template <int P, int R, int K, int LF = 0>
__device__ __forceinline__ void hop_site(const Geom &g, const LinkRef &L, int parity, const Site &s, int cb,
                                         const char *in, int64_t in_stride, const bool *active,
                                         V3<typename RealOf<P>::type> *acc, const char *win = nullptr,
                                         int win_stride = 0, int w0 = 0, int wlen = 0)
{
    typedef typename RealOf<P>::type T;
    if constexpr (P == F16) {
        hop_site_h<R, K, LF>(g, L, parity, s, cb, in, in_stride, active, acc, win, win_stride, w0, wlen);
        return;
    }
    constexpr bool TG = (LF & LF_TEMPORAL) != 0, NT = (LF & LF_STREAM) != 0;
    const char *lb = (const char *)L.base;
#pragma unroll
    for (int j = 0; j < K; ++j) acc[j] = vzero<T>();
    if constexpr ((LF & LF_PREFETCH) != 0) {
        // The compiler otherwise keeps a few loads in flight per wave (it
        // holds registers down for occupancy) and waits for each direction's
        // words before it asks for the next.  Here a group of directions has
        // all its words requested (the links and every right-hand side's
        // neighbour), a scheduling barrier keeps the decoding below them, and
        // the products accumulate in the order of the loop below (same bits).
        // Inactive right-hand sides load side 0's words and drop them, so that
        // no load sits behind a branch.  Groups: all eight directions for one
        // FP16/FP32 vector, four for two, two for four; FP64 four, then two.
        static_assert((LF & LF_LDS) == 0, "prefetch: no LDS window");
        typedef LinkIO<P, R, NT> LIO;
        constexpr int GRP = P == F64 ? (K == 1 ? 4 : 2) : (K == 1 ? 8 : K == 2 ? 4 : 2);
#pragma unroll
        for (int d0 = 0; d0 < 8; d0 += GRP) {
            typename LIO::Raw lr[GRP];
            typename SpinorIO<P>::Raw vr[GRP][K];
#pragma unroll
            for (int k = 0; k < GRP; ++k) {
                const int d = d0 + k, mu = d >> 1;
                const bool fwd = (d & 1) == 0;
                const bool unit = TG && mu == 3 && (s.tunit & (fwd ? 1u : 2u));
                const int at = unit ? g.vh : (fwd ? cb : s.bwd[mu]);
                lr[k] = LIO::load_raw(lb + (2 * mu + (fwd ? parity : 1 - parity)) * L.block_bytes, L.pitch, at);
#pragma unroll
                for (int j = 0; j < K; ++j)
                    vr[k][j] = SpinorIO<P>::load_raw(in + (active[j] ? j : 0) * in_stride, g.vh,
                                                     fwd ? s.fwd[mu] : s.bwd[mu]);
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int k = 0; k < GRP; ++k) {
                const int d = d0 + k, mu = d >> 1;
                const M3<T> u = LIO::decode(lr[k]);
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    if (!active[j]) continue;
                    const V3<T> v = SpinorIO<P>::decode(vr[k][j]);
                    if ((d & 1) == 0) accum(acc[j], mv(u, v), (s.negf >> mu) & 1);
                    else accum(acc[j], mdv(u, v), !((s.negb >> mu) & 1));
                }
            }
        }
        return;
    }
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const bool nf = (s.negf >> mu) & 1;
        const bool nb = !((s.negb >> mu) & 1);
        // temporal gauge (Sec. 4.3): the t-links are unit matrices except on
        // the last time slice; they are not read from the link arrays, the
        // unit link stored at index vh of the t-link blocks (always cached)
        // is read instead.  Selecting the site index keeps the code free of
        // branches (a branch around the product quadruples the register
        // count of this loop, a second base address doubles it).
        const bool uf_unit = TG && mu == 3 && (s.tunit & 1u);
        const bool ub_unit = TG && mu == 3 && (s.tunit & 2u);
        const M3<T> uf = LinkIO<P, R, NT>::load(lb + (2 * mu + parity) * L.block_bytes, L.pitch, uf_unit ? g.vh : cb);
#pragma unroll
        for (int j = 0; j < K; ++j) {
            if (!active[j]) continue;
            const int nbr = s.fwd[mu];
            const bool lw = (LF & LF_LDS) && mu < 2 && nbr >= w0 && nbr < w0 + wlen;
            const V3<T> v = lw ? SpinorIO<P>::load(win + j * win_stride, wlen, nbr - w0)
                               : SpinorIO<P>::load(in + j * in_stride, g.vh, nbr);
            accum(acc[j], mv(uf, v), nf);
        }
        const M3<T> ub = LinkIO<P, R, NT>::load(lb + (2 * mu + 1 - parity) * L.block_bytes, L.pitch,
                                                ub_unit ? g.vh : s.bwd[mu]);
#pragma unroll
        for (int j = 0; j < K; ++j) {
            if (!active[j]) continue;
            const int nbr = s.bwd[mu];
            const bool lw = (LF & LF_LDS) && mu < 2 && nbr >= w0 && nbr < w0 + wlen;
            const V3<T> v = lw ? SpinorIO<P>::load(win + j * win_stride, wlen, nbr - w0)
                               : SpinorIO<P>::load(in + j * in_stride, g.vh, nbr);
            accum(acc[j], mdv(ub, v), nb);
        }
    }
}

// Single right-hand side, input vectors produced by load(cb_neighbour) (for
// operands formed on the fly, e.g. r + beta p in the persistent solver).
template <int P, int R, typename Load>
__device__ __forceinline__ V3<typename RealOf<P>::type> hop_site_fn(const Geom &g, const LinkRef &L, int parity,
                                                                   const Site &s, int cb, Load load)
{
    typedef typename RealOf<P>::type T;
    const char *lb = (const char *)L.base;
    V3<T> acc = vzero<T>();
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const M3<T> uf = LinkIO<P, R>::load(lb + (2 * mu + parity) * L.block_bytes, L.pitch, cb);
        accum(acc, mv(uf, load(s.fwd[mu])), (s.negf >> mu) & 1);
        const M3<T> ub = LinkIO<P, R>::load(lb + (2 * mu + 1 - parity) * L.block_bytes, L.pitch, s.bwd[mu]);
        accum(acc, mdv(ub, load(s.bwd[mu])), !((s.negb >> mu) & 1));
    }
    return acc;
}

}  // namespace lqs
