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
// LF_STREAM, link words are fetched with streaming loads.  Inactive right-hand
// sides are skipped and keep acc = 0.  `in` points at right-hand side 0 of
// the input field (parity 1 - parity); consecutive sides are in_stride bytes
// apart.
enum { LF_TEMPORAL = 1, LF_STREAM = 2 };

// Block -> (site tile, right-hand-side group) for launches over several
// groups of right-hand sides.  The G blocks of one site tile are 8 block
// indices apart: the round-robin dispatch over the 8 XCDs puts them on the
// same XCD in close succession, so the links they share come from HBM once
// and then from that XCD's L2.  The grid has ceil(tiles / 8) * 8 * G blocks;
// tiles past the last are empty.  With G == 1 the map is the identity.
__device__ __forceinline__ void tile_group(int G, int &tile, int &grp)
{
    if (G == 1) {
        tile = blockIdx.x;
        grp = 0;
        return;
    }
    const int b = blockIdx.x, xcd = b & 7, q = b >> 3;
    grp = q % G;
    tile = (q / G) * 8 + xcd;
}

inline unsigned tile_group_blocks(int tiles, int G) { return G == 1 ? tiles : ((tiles + 7) / 8) * 8 * G; }

template <int P, int R, int K, int LF = 0>
__device__ __forceinline__ void hop_site(const Geom &g, const LinkRef &L, int parity, const Site &s, int cb,
                                         const char *in, int64_t in_stride, const bool *active,
                                         V3<typename RealOf<P>::type> *acc)
{
    typedef typename RealOf<P>::type T;
    constexpr bool TG = (LF & LF_TEMPORAL) != 0, NT = (LF & LF_STREAM) != 0;
    const char *lb = (const char *)L.base;
#pragma unroll
    for (int j = 0; j < K; ++j) acc[j] = vzero<T>();
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const bool nf = (s.negf >> mu) & 1;
        const bool nb = !((s.negb >> mu) & 1);
        // temporal gauge (Sec. 4.3): the t-links are unit matrices except on
        // the last time slice; they are not read from the link arrays, the
        // one stored unit link (vh = 1, always cached) is read instead.
        // Selecting the address keeps the code free of branches (a branch
        // around the product quadruples the register count of this loop).
        const bool uf_unit = TG && mu == 3 && (s.tunit & 1u);
        const bool ub_unit = TG && mu == 3 && (s.tunit & 2u);
        const M3<T> uf = LinkIO<P, R, NT>::load(uf_unit ? (const char *)L.unit : lb + (2 * mu + parity) * L.block_bytes,
                                                uf_unit ? 1 : g.vh, uf_unit ? 0 : cb);
#pragma unroll
        for (int j = 0; j < K; ++j) {
            if (!active[j]) continue;
            const V3<T> v = SpinorIO<P>::load(in + j * in_stride, g.vh, s.fwd[mu]);
            accum(acc[j], mv(uf, v), nf);
        }
        const M3<T> ub = LinkIO<P, R, NT>::load(ub_unit ? (const char *)L.unit
                                                        : lb + (2 * mu + 1 - parity) * L.block_bytes,
                                                ub_unit ? 1 : g.vh, ub_unit ? 0 : s.bwd[mu]);
#pragma unroll
        for (int j = 0; j < K; ++j) {
            if (!active[j]) continue;
            const V3<T> v = SpinorIO<P>::load(in + j * in_stride, g.vh, s.bwd[mu]);
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
        const M3<T> uf = LinkIO<P, R>::load(lb + (2 * mu + parity) * L.block_bytes, g.vh, cb);
        accum(acc, mv(uf, load(s.fwd[mu])), (s.negf >> mu) & 1);
        const M3<T> ub = LinkIO<P, R>::load(lb + (2 * mu + 1 - parity) * L.block_bytes, g.vh, s.bwd[mu]);
        accum(acc, mdv(ub, load(s.bwd[mu])), !((s.negb >> mu) & 1));
    }
    return acc;
}

}  // namespace lqs
