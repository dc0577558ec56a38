"""GPU CG against the oracle: FP64, mixed precision, multi-RHS, warm start.

The bar for every solve is the FP64 true residual ||b - M x|| / ||b|| <= tol,
recomputed by the CPU oracle on the GPU's x; the GPU's own FP64 residual
must agree with it, and x must agree with the oracle's solution to within
kappa * tol (kappa = condition number bound (m^2 + 64) / m^2, since
||D_eo D_oe|| <= 64).
"""
import numpy as np
import pytest

import oracle
import synth
from paper_2502_03249_amd import model
from gpu_util import field, gauge, lex_of, rel

pytestmark = pytest.mark.gpu

lqs = pytest.importorskip("paper_2502_03249_amd")


@pytest.fixture(scope="module")
def ctx():
    c = lqs.Context(0)
    yield c
    c.close()


def _solve(ctx, dims, U, mass, b, tol=1e-10, nrhs=1, **kw):
    g = gauge(ctx, dims, U)
    bf = field(ctx, dims, b, 0)
    xf = bf.like().zero_()
    stats = lqs.cg_solve(ctx, [(g, mass, bf, xf)], tol=tol, **kw)
    return lex_of(ctx, xf, squeeze=(nrhs == 1)), stats


def test_cg_fp64_config_4x4_haar(ctx):
    """4^4, Haar links (seed 1000), Gaussian even source (seed 2000), m = 0.1."""
    dims, mass = (4, 4, 4, 4), 0.1
    U = synth.gauge(dims, "haar", seed=1000)
    b = synth.source(dims, 0, seed=2000)
    x, st = _solve(ctx, dims, U, mass, b)
    assert st[0]["status"] == 0
    tr = oracle.true_residual(dims, U, mass, b, x)
    assert tr <= 1e-10 and abs(tr - st[0]["true_rel_residual"]) <= 1e-3 * tr + 1e-16
    xo, so, _, _ = oracle.cg(dims, U, mass, b)
    assert rel(x, xo) <= (mass ** 2 + 64) / mass ** 2 * 1e-10


def test_cg_fp64_config_32x8_smooth(ctx):
    """32^3 x 8, smooth links eps = 0.3 (seed 1001), Gaussian source (seed 2001), m = 0.02."""
    dims, mass = (32, 32, 32, 8), 0.02
    U = synth.gauge(dims, "smooth", seed=1001, eps=0.3)
    b = synth.source(dims, 0, seed=2001)
    x, st = _solve(ctx, dims, U, mass, b)
    assert st[0]["status"] == 0
    tr = oracle.true_residual(dims, U, mass, b, x)
    assert tr <= 1e-10 and abs(tr - st[0]["true_rel_residual"]) <= 1e-3 * tr + 1e-16
    assert np.abs(x * (np.indices(x.shape[:4]).sum(0) % 2 == 1)[..., None]).max() == 0.0
    xo, so, _, _ = oracle.cg(dims, U, mass, b)
    assert so == 0
    assert rel(x, xo) <= (mass ** 2 + 64) / mass ** 2 * 1e-10


@pytest.mark.parametrize("prec,recon", [(lqs.F32, 18), (lqs.F16, 18), (lqs.F32, 12), (lqs.F16, 12)])
def test_cg_mixed_precision_reaches_fp64_residual(ctx, prec, recon):
    dims, mass = (16, 16, 16, 8), 0.02
    U = synth.gauge(dims, "smooth", seed=41, eps=0.3)
    b = synth.source(dims, 0, seed=42)
    x, st = _solve(ctx, dims, U, mass, b, inner_prec=prec, inner_recon=recon, reliable_interval=100)
    assert st[0]["status"] == 0, st
    assert st[0]["reliable_updates"] >= 1
    assert oracle.true_residual(dims, U, mass, b, x) <= 1e-10
    xo, _, _, _ = oracle.cg(dims, U, mass, b)
    assert rel(x, xo) <= (mass ** 2 + 64) / mass ** 2 * 1e-10
    # reported rates: 1140 flop and the model's algorithmic bytes per even site and iteration
    s0 = st[0]
    n = np.prod(dims) // 2 * s0["iters"]
    assert s0["device_seconds"] > 0
    assert s0["gflops"] == pytest.approx(1140 * n / s0["device_seconds"] * 1e-9, rel=1e-12)
    want_b = model.cg_iteration_bytes(prec, lqs.F32, recon) * n / s0["device_seconds"] * 1e-9
    assert s0["gbytes_per_s"] == pytest.approx(want_b, rel=1e-12)


@pytest.mark.parametrize("prec", [lqs.F64, lqs.F32, lqs.F16])
def test_cg_multi_rhs_each_column(ctx, prec):
    """nrhs independent CGs sharing the links: every column reaches the residual on its own."""
    dims, mass, nrhs = (8, 8, 8, 8), 0.05, 5
    U = synth.gauge(dims, "smooth", seed=51, eps=0.3)
    bs = np.stack([synth.source(dims, 0, seed=5100 + k) for k in range(nrhs)])
    bs[2] *= 1e-3   # columns of very different norm converge at different iterations
    x, st = _solve(ctx, dims, U, mass, bs, nrhs=nrhs, inner_prec=prec, reliable_interval=50)
    assert len(st) == nrhs
    for k in range(nrhs):
        assert st[k]["status"] == 0
        assert oracle.true_residual(dims, U, mass, bs[k], x[k]) <= 1e-10


@pytest.mark.parametrize("prec", [lqs.F64, lqs.F32, lqs.F16])
def test_cg_block_with_zero_and_point_sources(ctx, prec):
    """A block of four columns on a ragged lattice: a Gaussian source, an all-zero source (that
    column is done at the start, x = 0 exactly), a point source (one colour at one even site, so
    at the start every other site of the FP16 vectors has scale zero) and a second Gaussian
    source.  Every column is reported converged and meets tol by the oracle's residual; the
    point-source solution agrees with the oracle's within the condition bound."""
    dims, mass = (4, 6, 8, 10), 0.1
    U = synth.gauge(dims, "haar", seed=61)
    bs = np.stack([synth.source(dims, 0, seed=6100 + k) for k in range(4)])
    bs[1] = 0.0
    bs[2] = 0.0
    bs[2][0, 0, 0, 0, 0] = 1.0  # site (x, y, z, t) = 0: even
    x, st = _solve(ctx, dims, U, mass, bs, nrhs=4, inner_prec=prec)
    assert [s["status"] for s in st] == [0, 0, 0, 0], st
    assert st[1]["iters"] == 0 and np.abs(x[1]).max() == 0.0
    for k in (0, 2, 3):
        assert oracle.true_residual(dims, U, mass, bs[k], x[k]) <= 1e-10, k
    xo, _, _, _ = oracle.cg(dims, U, mass, bs[2], tol=1e-11)
    assert rel(x[2], xo) <= (mass ** 2 + 64) / mass ** 2 * 1e-10


def test_cg_warm_start_resume(ctx):
    dims, mass = (8, 8, 8, 8), 0.05
    U = synth.gauge(dims, "haar", seed=61)
    b = synth.source(dims, 0, seed=62)
    g = gauge(ctx, dims, U)
    bf = field(ctx, dims, b, 0)
    xf = bf.like().zero_()
    s1 = lqs.cg_solve(ctx, [(g, mass, bf, xf)], tol=1e-5)
    assert s1[0]["status"] == 0 and s1[0]["true_rel_residual"] <= 1e-5
    s2 = lqs.cg_solve(ctx, [(g, mass, bf, xf)], tol=1e-10, use_x0=True)
    assert s2[0]["status"] == 0
    x = lex_of(ctx, xf)
    assert oracle.true_residual(dims, U, mass, b, x) <= 1e-10


@pytest.mark.parametrize("dims,mass,tol", [((4, 4, 4, 4), 0.1, 1e-13), ((8, 8, 8, 8), 0.05, 1e-12)])
def test_cg_fp64_restart_near_rounding_limit(ctx, dims, mass, tol):
    """An FP64 solve to a tolerance near the rounding limit: the iterated residual meets tol
    before the true one does, so the FP64 check restarts CG from r = b - M x (beta = 0) at least
    once.  That path applies the pending x step in the FP64 group before the check and skips it
    in the p-update after; the solution must still meet tol by the oracle's residual, and the
    GPU's own FP64 residual must agree with it."""
    U = synth.gauge(dims, "haar", seed=61)
    b = synth.source(dims, 0, seed=62)
    g = gauge(ctx, dims, U)
    bf = field(ctx, dims, b, 0)
    xf = bf.like().zero_()
    st = lqs.cg_solve(ctx, [(g, mass, bf, xf)], tol=tol, max_iter=20000)[0]
    assert st["status"] == 0 and st["restarts"] >= 1, st
    tr = oracle.true_residual(dims, U, mass, b, lex_of(ctx, xf))
    assert tr <= tol
    assert abs(tr - st["true_rel_residual"]) <= 0.05 * tr


def test_cg_max_iter_reports_not_converged(ctx):
    dims, mass = (4, 4, 4, 4), 0.1
    U = synth.gauge(dims, "haar", seed=1000)
    b = synth.source(dims, 0, seed=2000)
    x, st = _solve(ctx, dims, U, mass, b, max_iter=7)
    assert st[0]["status"] == lqs.ENOTCONV
    assert st[0]["iters"] >= 7
    tr = oracle.true_residual(dims, U, mass, b, x)
    assert abs(tr - st[0]["true_rel_residual"]) <= 1e-6 * tr


def test_cg_zero_source(ctx):
    dims = (4, 4, 4, 4)
    U = synth.gauge(dims, "haar", seed=1)
    b = np.zeros((4, 4, 4, 4, 3), np.complex128)
    x, st = _solve(ctx, dims, U, 0.1, b)
    assert st[0]["status"] == 0 and np.abs(x).max() == 0.0


def test_cg_full_size_benchmark_solve(ctx):
    """The timed solve at full size: 64^3 x 16, m = 0.01, FP16 12-real inner, reliable updates every
    100 iterations; the oracle recomputes ||b - M x|| / ||b|| in FP64."""
    dims, mass = (64, 64, 64, 16), 0.01
    U = synth.gauge(dims, "smooth", seed=1002, eps=0.3)
    b = synth.source(dims, 0, seed=2002)
    g = gauge(ctx, dims, U)
    bf = field(ctx, dims, b, 0)
    xf = bf.like().zero_()
    st = lqs.cg_solve(ctx, [(g, mass, bf, xf)], tol=1e-10, inner_prec=lqs.F16, inner_recon=12,
                      reliable_interval=100)
    assert st[0]["status"] == 0
    x = lex_of(ctx, xf)
    tr = oracle.true_residual(dims, U, mass, b, x)
    assert tr <= 1e-10
    assert abs(tr - st[0]["true_rel_residual"]) <= 1e-12


def test_cg_full_size_sixteen_rhs(ctx):
    """The largest block of independent solves at full size: 64^3 x 16, 16 right-hand sides,
    FP32 12-real inner with FP64 reliable updates; the oracle recomputes the FP64 true residual
    of sampled columns."""
    dims, mass, nrhs = (64, 64, 64, 16), 0.01, 16
    U = synth.gauge(dims, "smooth", seed=1002, eps=0.3)
    b = np.stack([synth.source(dims, 0, seed=2300 + k) for k in range(nrhs)])
    g = gauge(ctx, dims, U, lqs.fmt(lqs.F64, 18) | lqs.fmt(lqs.F64, 12) | lqs.fmt(lqs.F32, 12))
    bf = field(ctx, dims, b, 0)
    xf = bf.like().zero_()
    st = lqs.cg_solve(ctx, [(g, mass, bf, xf)], tol=1e-10, inner_prec=lqs.F32, inner_recon=12,
                      reliable_interval=100)
    assert len(st) == nrhs and all(s["status"] == 0 for s in st)
    x = lex_of(ctx, xf, squeeze=False)
    for k in (0, 9, nrhs - 1):
        tr = oracle.true_residual(dims, U, mass, b[k], x[k])
        assert tr <= 1e-10, (k, tr)
        assert abs(tr - st[k]["true_rel_residual"]) <= 1e-12, k


@pytest.mark.parametrize("prec,recon,nrhs", [(lqs.F64, 18, 1), (lqs.F16, 12, 1), (lqs.F32, 12, 3)])
def test_graph_replay_equals_eager(ctx, prec, recon, nrhs):
    """Solves whose iteration rounds are captured once into a HIP graph and replayed (with the
    host's polls and copies between the replays) give the same bits and iteration counts as
    launching every kernel; a second solve in a row recaptures for its own buffers."""
    dims, mass = (8, 8, 8, 16), 0.05
    U = synth.gauge(dims, "smooth", seed=131, eps=0.3)
    b = np.stack([synth.source(dims, 0, seed=1310 + k) for k in range(nrhs)])
    g = gauge(ctx, dims, U)
    out = {}
    for graphs in (False, True):
        ctx.set_graphs(graphs)
        for rep in range(2):
            bf = field(ctx, dims, b, 0)
            xf = bf.like().zero_()
            st = lqs.cg_solve(ctx, [(g, mass, bf, xf)], tol=1e-10, inner_prec=prec, inner_recon=recon,
                              reliable_interval=50)
            assert all(s["status"] == 0 for s in st)
            out[(graphs, rep)] = (lex_of(ctx, xf, squeeze=False), [s["iters"] for s in st])
    ctx.set_graphs(True)
    ref = out[(False, 0)]
    for k, (x, its) in out.items():
        assert its == ref[1], k
        assert np.array_equal(x, ref[0]), k
    for k in range(nrhs):
        assert oracle.true_residual(dims, U, mass, b[k], ref[0][k]) <= 1e-10


@pytest.mark.parametrize("prec", [lqs.F16, lqs.F32])
def test_reliable_updates_every_chunk_hand_off_to_the_18_real_check(ctx, prec):
    """A 12-real mixed solve with a reliable update due at every opportunity: the periodic
    updates run on the FP64 12-real links. Near the end one of them meets the target and hands
    the solve, still pending, to the check on the stored 18-real links. The check alone declares
    convergence, and the reported residual agrees with the oracle's on the original links."""
    dims, mass = (8, 8, 8, 16), 0.05
    U = synth.gauge(dims, "smooth", seed=141, eps=0.3)
    b = synth.source(dims, 0, seed=142)
    for delta in (0.9, 0.0):
        x, st = _solve(ctx, dims, U, mass, b, inner_prec=prec, inner_recon=12, reliable_interval=1,
                       reliable_delta=delta)
        assert st[0]["status"] == 0, st
        assert st[0]["reliable_updates"] >= 10
        tr = oracle.true_residual(dims, U, mass, b, x)
        assert tr <= 1e-10
        assert abs(tr - st[0]["true_rel_residual"]) <= 1e-13
