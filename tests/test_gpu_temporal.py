"""Temporal gauge (the paper's 6-link storage): gauge fixing, the hop that skips
unit t-links, and a solve in the fixed gauge mapped back by G."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import dev, field, gauge, host, lex_of, rel
from latt import apply_site, gauge_transform

pytestmark = pytest.mark.gpu

lqs = pytest.importorskip("paper_2502_03249_amd")


@pytest.fixture(scope="module")
def ctx():
    c = lqs.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("dims", [(4, 6, 8, 10), (8, 8, 8, 16)])
def test_gauge_fixing(ctx, dims):
    U = synth.gauge(dims, "haar", seed=111)
    Uf, G = lqs.gauge_fix_temporal(ctx, dims, dev(U))
    Uf, G = host(Uf), host(G)
    nt = dims[3]
    eye = np.eye(3)
    assert np.array_equal(Uf[3, :nt - 1], np.broadcast_to(eye, Uf[3, :nt - 1].shape))
    # G is SU(3) and the transformed links are G U G^dag (t-links of the last slice included)
    assert np.abs(G @ np.conj(np.swapaxes(G, -1, -2)) - eye).max() < 1e-13
    assert np.abs(np.linalg.det(G) - 1).max() < 1e-13
    want = gauge_transform(U, G)
    assert rel(Uf[:3], want[:3]) < 1e-13
    assert rel(Uf[3, nt - 1], want[3, nt - 1]) < 1e-13
    assert np.abs(want[3, :nt - 1] - eye).max() < 1e-12


@pytest.mark.parametrize("prec,recon,bound", [(lqs.F64, 18, 1e-12), (lqs.F64, 12, 1e-12), (lqs.F32, 12, 2e-6),
                                              (lqs.F16, 12, 4e-3)])
def test_temporal_hop_matches_oracle(ctx, prec, recon, bound):
    """The hop on the gauge-fixed links with the t-link reads skipped equals eq. (1) on those links."""
    dims = (4, 6, 8, 10)
    U = synth.gauge(dims, "haar", seed=112)
    Uf = host(lqs.gauge_fix_temporal(ctx, dims, dev(U))[0])
    src = synth.source(dims, -1, seed=113)
    g = lqs.Gauge(ctx, dims, dev(Uf), lqs.FMT_ALL | lqs.TEMPORAL_GAUGE)
    for out_parity in (0, 1):
        x = field(ctx, dims, src, 1 - out_parity, prec)
        got = lex_of(ctx, lqs.dslash_apply(ctx, g, x, recon=recon))
        assert rel(got, oracle.dslash(dims, Uf, src, out_parity)) <= bound


def test_temporal_flag_rejects_unfixed_links(ctx):
    dims = (4, 4, 4, 4)
    U = synth.gauge(dims, "haar", seed=114)
    with pytest.raises(lqs.LqsError) as e:
        lqs.Gauge(ctx, dims, dev(U), lqs.FMT_ALL | lqs.TEMPORAL_GAUGE)
    assert e.value.status == lqs.EINVAL


def test_solve_in_temporal_gauge_maps_back(ctx):
    """M[U'] (G x) = G M[U] x: solving with G b in the fixed gauge and applying G^dag gives M[U]^-1 b."""
    dims, mass = (8, 8, 8, 8), 0.05
    U = synth.gauge(dims, "smooth", seed=115, eps=0.3)
    b = synth.source(dims, 0, seed=116)
    Uf_d, G_d = lqs.gauge_fix_temporal(ctx, dims, dev(U))
    G = host(G_d)
    g = lqs.Gauge(ctx, dims, Uf_d, lqs.FMT_ALL | lqs.TEMPORAL_GAUGE)
    bf = field(ctx, dims, apply_site(G, b), 0)
    xf = bf.like().zero_()
    st = lqs.cg_solve(ctx, [(g, mass, bf, xf)], tol=1e-10, inner_prec=lqs.F16, inner_recon=12,
                      reliable_interval=100)
    assert st[0]["status"] == 0
    x = apply_site(np.conj(np.swapaxes(G, -1, -2)), lex_of(ctx, xf))
    # U' equals G U G^dag to ~1e-16 per entry, so ||b - M x|| / ||b|| differs from the
    # fixed-gauge residual by at most ~1e-16 * ||M|| ||x|| / ||b|| <= 1e-16 * 64 / m^2 = 2.6e-12
    assert oracle.true_residual(dims, U, mass, b, x) <= 1e-10 + 3e-12


@pytest.mark.parametrize("prec,recon,nrhs,bound", [(lqs.F64, 18, 3, 1e-12), (lqs.F32, 12, 5, 2e-6),
                                                   (lqs.F16, 12, 2, 4e-3), (lqs.F64, 12, 1, 1e-12)])
def test_temporal_hop_multi_rhs_and_dagger(ctx, prec, recon, nrhs, bound):
    """Several right-hand sides per link read (one, two and four per thread, groups with an
    inactive side) and the dagger, on a lattice whose 96-site time slices split wavefronts,
    so that unit and stored t-links meet inside one wavefront."""
    dims = (4, 6, 8, 10)
    U = synth.gauge(dims, "haar", seed=117)
    Uf = host(lqs.gauge_fix_temporal(ctx, dims, dev(U))[0])
    g = lqs.Gauge(ctx, dims, dev(Uf), lqs.FMT_ALL | lqs.TEMPORAL_GAUGE)
    srcs = np.stack([synth.source(dims, 1, seed=1170 + k) for k in range(nrhs)])
    x = field(ctx, dims, srcs, 1, prec)
    got = lex_of(ctx, lqs.dslash_apply(ctx, g, x, recon=recon), squeeze=False)
    gotd = lex_of(ctx, lqs.dslash_dagger(ctx, g, x, recon=recon), squeeze=False)
    for k in range(nrhs):
        want = oracle.dslash(dims, Uf, srcs[k], 0)
        assert rel(got[k], want) <= bound
        assert rel(gotd[k], oracle.dslash_dagger(dims, Uf, srcs[k], 0)) <= bound
