"""GPU hop parity against the CPU oracle (element by element, through the C ABI).

Sizes span several 256-thread blocks and ragged tails (4x6x8x10 has Vh = 960,
not a multiple of 256); 32^3x8 and 64^3x16 are the benchmark lattices, run in
the launch configuration the benchmark uses.
FP64 bar: relative L2 error <= 1e-12.  FP32 / FP16-storage bars: a relative L2
error of a few unit roundoffs, and at every output site an error of at most
SITE_C unit roundoffs times the summed norms of its eight input neighbours
(see test_hop_low_precision and gpu_util.site_error_ratio).
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import U_F16, U_F32, dev, field, gauge, host, lex_of, rel, site_error_ratio

pytestmark = pytest.mark.gpu

lqs = pytest.importorskip("paper_2502_03249_amd")


@pytest.fixture(scope="module")
def ctx():
    c = lqs.Context(0)
    yield c
    c.close()


# Per-site bound in unit roundoffs.  Per neighbour term: the rounded link
# changes U v by at most |dU|_F |v| <= sqrt(18) u |v| (the rebuilt third row of
# a 12-real link adds about 2 u per entry), the rounded vector (six components
# scaled by the site's largest) by sqrt(6) u |v|; the output rounding adds
# sqrt(6) u times the largest output component.  In the worst alignment that
# is under 10 u per unit of summed neighbour norm; FP32 accumulation adds
# about 11 u_f32.  16 leaves a margin; one wrong site gives a ratio near 1.
SITE_C = 16


def _case(dims, kind, seed):
    U = synth.gauge(dims, kind, seed=seed, eps=0.3)
    src = synth.source(dims, -1, seed=seed + 1)
    return U, src


@pytest.mark.parametrize("dims,kind", [((4, 4, 4, 4), "haar"), ((4, 6, 8, 10), "haar"), ((2, 4, 2, 6), "haar"),
                                       ((8, 8, 8, 8), "smooth"), ((32, 32, 32, 8), "smooth")])
@pytest.mark.parametrize("recon", [18, 12])
@pytest.mark.parametrize("out_parity", [0, 1])
def test_hop_f64_matches_oracle(ctx, dims, kind, recon, out_parity):
    U, src = _case(dims, kind, 100 + dims[3])
    g = gauge(ctx, dims, U)
    x = field(ctx, dims, src, 1 - out_parity)
    y = lqs.dslash_apply(ctx, g, x, recon=recon)
    got = lex_of(ctx, y)
    want = oracle.dslash(dims, U, src, out_parity)
    assert rel(got, want) <= 1e-12


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (4, 6, 8, 10)])
@pytest.mark.parametrize("out_parity", [0, 1])
def test_dagger_matches_oracle_adjoint(ctx, dims, out_parity):
    """The separate adjoint kernel against the oracle's conjugate-transpose stencil."""
    U, src = _case(dims, "haar", 7)
    g = gauge(ctx, dims, U)
    x = field(ctx, dims, src, 1 - out_parity)
    got = lex_of(ctx, lqs.dslash_dagger(ctx, g, x))
    want = oracle.dslash_dagger(dims, U, src * (np.indices(src.shape[:4]).sum(0) % 2 == 1 - out_parity)[..., None],
                                out_parity)
    assert rel(got, want) <= 1e-12


@pytest.mark.parametrize("prec,recon,bound", [(lqs.F32, 18, 2e-6), (lqs.F32, 12, 2e-6), (lqs.F16, 18, 4e-3),
                                              (lqs.F16, 12, 4e-3)])
def test_hop_low_precision(ctx, prec, recon, bound):
    """FP32 / FP16-storage hops against the FP64 oracle on the same inputs.

    Each output sums 8 SU(3) products of 3 terms; rounding the inputs to the
    storage precision (unit roundoff u = 6e-8 for FP32, 4.9e-4 for binary16)
    and accumulating in FP32 gives a relative L2 error of order a few u; the
    bounds allow about 8 u (FP32 also covers the FP32 accumulation).
    """
    dims = (8, 8, 8, 16)
    U, src = _case(dims, "smooth", 31)
    g = gauge(ctx, dims, U)
    x = field(ctx, dims, src, 1, prec)
    got = lex_of(ctx, lqs.dslash_apply(ctx, g, x, recon=recon))
    want = oracle.dslash(dims, U, src, 0)
    err = rel(got, want)
    assert err <= bound, err
    u = U_F16 if prec == lqs.F16 else U_F32
    ratio = site_error_ratio(dims, got, want, src, 0)
    assert ratio <= SITE_C * u, (ratio / u)


@pytest.mark.parametrize("prec", [lqs.F64, lqs.F32, lqs.F16])
@pytest.mark.parametrize("nrhs", [2, 3, 5, 16])
def test_multi_rhs_columns_equal_single(ctx, prec, nrhs):
    """The multi-vector hop reads each link once; column k equals the single-vector hop bit for bit."""
    dims = (4, 6, 8, 10)
    U = synth.gauge(dims, "haar", seed=5)
    srcs = np.stack([synth.source(dims, -1, seed=500 + k) for k in range(nrhs)])
    g = gauge(ctx, dims, U)
    xm = field(ctx, dims, srcs, 1, prec)
    ym = lex_of(ctx, lqs.dslash_apply(ctx, g, xm), squeeze=False)
    for k in range(nrhs):
        xs = field(ctx, dims, srcs[k], 1, prec)
        ys = lex_of(ctx, lqs.dslash_apply(ctx, g, xs))
        assert np.array_equal(ym[k], ys)
    if prec == lqs.F64:
        want = oracle.dslash(dims, U, srcs[nrhs - 1], 0)
        assert rel(ym[nrhs - 1], want) <= 1e-12


def test_pack_layout_matches_header(ctx):
    """The native FP64 layout is double2 [3][Vh] with cb = lex >> 1 (checked in numpy, not by the library)."""
    dims = (4, 6, 8, 10)
    src = synth.source(dims, -1, seed=9)
    for parity in (0, 1):
        f = field(ctx, dims, src, parity)
        raw = host(f.data).view(np.float64)
        vh = np.prod(dims) // 2
        want = np.zeros((3, vh), np.complex128)
        flat = src.reshape(-1, 3)
        nx, ny, nz, nt = dims
        for lex in range(np.prod(dims)):
            x, y, z, t = lex % nx, (lex // nx) % ny, (lex // (nx * ny)) % nz, lex // (nx * ny * nz)
            if (x + y + z + t) % 2 == parity:
                want[:, lex >> 1] = flat[lex]
        got = raw.reshape(3, vh, 2)
        assert np.array_equal(got[..., 0], want.real) and np.array_equal(got[..., 1], want.imag)


def test_unpack_roundtrip_and_parity_isolation(ctx):
    dims = (4, 4, 6, 8)
    src = synth.source(dims, -1, seed=10)
    for prec, tol in ((lqs.F64, 0.0), (lqs.F32, 1e-7), (lqs.F16, 1e-3)):
        f = field(ctx, dims, src, 1, prec)
        back = lex_of(ctx, f)
        odd = src * (np.indices(src.shape[:4]).sum(0) % 2 == 1)[..., None]
        assert np.abs(back - odd).max() <= tol * np.abs(src).max()


def test_full_size_hop_64x16(ctx):
    """64^3 x 16, smooth links (eps = 0.3, seed 1002), FP64 18 and 12 reals: the benchmark's hop."""
    dims = (64, 64, 64, 16)
    U = synth.gauge(dims, "smooth", seed=1002, eps=0.3)
    src = synth.source(dims, 1, seed=2002)
    g = gauge(ctx, dims, U, lqs.fmt(lqs.F64, 18) | lqs.fmt(lqs.F64, 12))
    x = field(ctx, dims, src, 1)
    want = oracle.dslash(dims, U, src, 0)
    for recon in (18, 12):
        got = lex_of(ctx, lqs.dslash_apply(ctx, g, x, recon=recon))
        assert rel(got, want) <= 1e-12


def test_full_size_low_precision_hops_64x16(ctx):
    """64^3 x 16: the FP16 12-real hop the timed solve runs, and FP32 12-real, against the oracle,
    in the launch configuration of the timed solve (default shape, streaming link loads); every
    output site is held to the per-site rounding bound, not only the global norm."""
    dims = (64, 64, 64, 16)
    U = synth.gauge(dims, "smooth", seed=1002, eps=0.3)
    src = synth.source(dims, 1, seed=2002)
    g = gauge(ctx, dims, U, lqs.fmt(lqs.F16, 12) | lqs.fmt(lqs.F32, 12) | lqs.fmt(lqs.F16, 18))
    want = oracle.dslash(dims, U, src, 0)
    for prec, recon, bound, u in ((lqs.F16, 12, 4e-3, U_F16), (lqs.F32, 12, 2e-6, U_F32),
                                  (lqs.F16, 18, 4e-3, U_F16)):
        print(f"64^3x16 hop prec={prec} recon={recon}", flush=True)
        got = lex_of(ctx, lqs.dslash_apply(ctx, g, field(ctx, dims, src, 1, prec), recon=recon))
        assert rel(got, want) <= bound
        ratio = site_error_ratio(dims, got, want, src, 0)
        assert ratio <= SITE_C * u, (prec, recon, ratio / u)
        del got


def test_full_size_sixteen_rhs_hop_64x16(ctx):
    """64^3 x 16 with 16 right-hand sides (1.6 GB of FP64 input, several groups of vectors per
    site tile): sampled columns equal the single-vector hop bit for bit and match the oracle."""
    dims, nrhs = (64, 64, 64, 16), 16
    U = synth.gauge(dims, "smooth", seed=1002, eps=0.3)
    srcs = np.stack([synth.source(dims, 1, seed=2200 + k) for k in range(nrhs)])
    g = gauge(ctx, dims, U, lqs.fmt(lqs.F64, 18) | lqs.fmt(lqs.F32, 12))
    want = {k: oracle.dslash(dims, U, srcs[k], 0) for k in (0, nrhs - 1)}
    for prec, recon, bound in ((lqs.F64, 18, 1e-12), (lqs.F32, 12, 2e-6)):
        print(f"16-rhs hop 64^3x16 prec={prec} recon={recon}", flush=True)
        ym = lex_of(ctx, lqs.dslash_apply(ctx, g, field(ctx, dims, srcs, 1, prec), recon=recon), squeeze=False)
        for k in (0, 7, nrhs - 1):
            ys = lex_of(ctx, lqs.dslash_apply(ctx, g, field(ctx, dims, srcs[k], 1, prec), recon=recon))
            assert np.array_equal(ym[k], ys), k
        for k, w in want.items():
            assert rel(ym[k], w) <= bound, (prec, k)
            if prec == lqs.F32:
                ratio = site_error_ratio(dims, ym[k], w, srcs[k], 0)
                assert ratio <= SITE_C * U_F32, (k, ratio / U_F32)
        del ym
