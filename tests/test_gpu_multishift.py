"""Multi-mass (multi-shift) CG against one oracle CG per mass."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import field, gauge, lex_of, rel

pytestmark = pytest.mark.gpu

lqs = pytest.importorskip("paper_2502_03249_amd")


@pytest.fixture(scope="module")
def ctx():
    c = lqs.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("dims,kind,masses", [((4, 6, 8, 10), "haar", [0.3, 0.1, 0.5, 1.0]),
                                              ((16, 16, 16, 8), "smooth", [0.02, 0.05, 0.1, 0.2, 0.4, 0.8]),
                                              ((4, 4, 4, 4), "haar", [0.2])])
def test_multishift_matches_separate_solves(ctx, dims, kind, masses):
    U = synth.gauge(dims, kind, seed=101, eps=0.3)
    b = synth.source(dims, 0, seed=102)
    g = gauge(ctx, dims, U)
    bf = field(ctx, dims, b, 0)
    xs = [bf.like() for _ in masses]
    st = lqs.cg_solve_multishift(ctx, g, masses, bf, xs, tol=1e-10)
    base_iters = max(s["iters"] for s in st)
    for m, x, s in zip(masses, xs, st):
        assert s["status"] == 0, s
        # the FP64 recurrence alone brings every mass to tol: no refinement CG ran (a lost
        # x_i += alpha_i p_i anywhere in the recurrence would leave that mass above tol)
        assert s["restarts"] == 0, s
        xv = lex_of(ctx, x)
        assert oracle.true_residual(dims, U, m, b, xv) <= 1e-10
        xo, _, _, _ = oracle.cg(dims, U, m, b, tol=1e-11)
        assert rel(xv, xo) <= (m ** 2 + 64) / m ** 2 * 1e-10
    # heavier masses converge in fewer shared iterations
    order = np.argsort(masses)
    iters = [st[i]["iters"] - 0 for i in order]
    assert iters[0] == base_iters


def test_multishift_argument_errors(ctx):
    """No persistent form (LQS_EUNSUPPORTED); an unknown precision or aliased solutions are LQS_EINVAL."""
    dims = (4, 4, 4, 4)
    g = gauge(ctx, dims, synth.gauge(dims, "haar", seed=1))
    bf = field(ctx, dims, synth.source(dims, 0, seed=2), 0)
    xs = [bf.like(), bf.like()]
    import ctypes
    m = (ctypes.c_double * 2)(0.1, 0.2)
    ptrs = (ctypes.c_void_p * 2)(*[x.data.data_ptr() for x in xs])
    stats = (lqs.LqsCgStats * 2)()

    def call(prm, p=ptrs):
        return lqs.lib().cg_solve_multishift(ctx.handle, g.handle, 2, m, ctypes.c_void_p(bf.data.data_ptr()), p,
                                             ctypes.byref(prm), stats, None)

    assert call(lqs.LqsCgParams(1e-10, 100, lqs.F32, 18, 0, 0.0, 0, 1)) == lqs.EUNSUPPORTED
    assert call(lqs.LqsCgParams(1e-10, 100, 3, 18, 0, 0.0, 0, 0)) == lqs.EINVAL
    ptrs2 = (ctypes.c_void_p * 2)(xs[0].data.data_ptr(), xs[0].data.data_ptr())
    assert call(lqs.LqsCgParams(1e-10, 100, lqs.F64, 18, 0, 0.0, 0, 0), ptrs2) == lqs.EINVAL


@pytest.mark.parametrize("prec,recon", [(lqs.F32, 12), (lqs.F16, 12), (lqs.F32, 18)])
def test_multishift_mixed_precision(ctx, prec, recon):
    """Recurrence with FP32 / FP16-storage search directions and operator, solutions accumulated
    in FP64, then per-mass FP64 checks with mixed-precision refinement: every mass reaches the
    FP64 true residual against the oracle."""
    dims, masses = (16, 16, 16, 8), [0.02, 0.05, 0.1, 0.4, 1.5]
    U = synth.gauge(dims, "smooth", seed=103, eps=0.3)
    b = synth.source(dims, 0, seed=104)
    g = gauge(ctx, dims, U)
    bf = field(ctx, dims, b, 0)
    xs = [bf.like() for _ in masses]
    st = lqs.cg_solve_multishift(ctx, g, masses, bf, xs, tol=1e-10, inner_prec=prec, inner_recon=recon)
    for m, x, s in zip(masses, xs, st):
        assert s["status"] == 0, s
        xv = lex_of(ctx, x)
        assert oracle.true_residual(dims, U, m, b, xv) <= 1e-10
        assert abs(oracle.true_residual(dims, U, m, b, xv) - s["true_rel_residual"]) <= 1e-12


@pytest.mark.parametrize("prec,recon", [(lqs.F64, 18), (lqs.F32, 12)])
def test_multishift_seventeen_masses_with_a_repeated_base(ctx, prec, recon):
    """The largest mass count (17: the base and 16 shifts, so the refinement runs as a block of
    16 columns and a block of one), with the smallest mass given twice: the repeated mass is a
    shift of zero, whose recurrence is the base's own.  Every mass meets tol by the oracle's
    residual and its solution agrees with the oracle's within the condition bound; the two
    copies of the base mass agree with each other (to rounding in FP64).  An 18th mass is rejected."""
    dims = (4, 6, 8, 10)  # 960 sites per parity: ragged 256-site tiles
    masses = [0.3, 0.3] + [0.35 + 0.1 * k for k in range(15)]
    assert len(masses) == 17
    U = synth.gauge(dims, "haar", seed=105)
    b = synth.source(dims, 0, seed=106)
    g = gauge(ctx, dims, U)
    bf = field(ctx, dims, b, 0)
    xs = [bf.like() for _ in masses]
    st = lqs.cg_solve_multishift(ctx, g, masses, bf, xs, tol=1e-10, inner_prec=prec, inner_recon=recon)
    sols = []
    for m, x, s in zip(masses, xs, st):
        assert s["status"] == 0, (m, s)
        xv = lex_of(ctx, x)
        assert oracle.true_residual(dims, U, m, b, xv) <= 1e-10, m
        xo, _, _, _ = oracle.cg(dims, U, m, b, tol=1e-11)
        assert rel(xv, xo) <= (m ** 2 + 64) / m ** 2 * 1e-10, m
        sols.append(xv)
    # FP64: the zero shift repeats the base's arithmetic; mixed: each copy is within the bound
    kappa = (masses[0] ** 2 + 64) / masses[0] ** 2
    assert rel(sols[1], sols[0]) <= (1e-12 if prec == lqs.F64 else 2 * kappa * 1e-10)
    with pytest.raises(lqs.LqsError):
        lqs.cg_solve_multishift(ctx, g, masses + [2.0], bf, xs + [bf.like()], tol=1e-10)
