"""torch.autograd Functions: gradcheck and parity with the oracle's derivatives."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import dev, host, rel

pytestmark = pytest.mark.gpu

lqs = pytest.importorskip("paper_2502_03249_amd")
from paper_2502_03249_amd.autograd import staggered_action, staggered_solve  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = lqs.Context(0)
    yield c
    c.close()


def _even(dims, seed):
    return synth.source(dims, 0, seed=seed)


def test_action_value_and_gradients_match_oracle(ctx):
    dims, mass = (4, 6, 8, 10), 0.2
    U = synth.gauge(dims, "haar", seed=81)
    phi = _even(dims, 82)
    Ut = dev(U).requires_grad_(True)
    pt = dev(phi).requires_grad_(True)
    S = staggered_action(Ut, pt, mass, ctx, project=False)
    S.backward()
    chi, st, _, _ = oracle.cg(dims, U, mass, phi, tol=1e-13)
    assert st == 0
    S_o = np.vdot(phi, chi).real
    assert abs(float(S) - S_o) <= 1e-10 * abs(S_o)
    assert rel(host(pt.grad), 2 * chi) <= 1e-9
    assert rel(host(Ut.grad), oracle.force(dims, U, chi, mode=1)) <= 1e-9


def test_action_projected_force_matches_oracle(ctx):
    dims, mass = (4, 4, 4, 8), 0.1
    U = synth.gauge(dims, "smooth", seed=83, eps=0.3)
    phi = _even(dims, 84)
    Ut = dev(U).requires_grad_(True)
    S = staggered_action(Ut, dev(phi), mass, ctx, project=True)
    (2.5 * S).backward()
    chi, _, _, _ = oracle.cg(dims, U, mass, phi, tol=1e-13)
    assert rel(host(Ut.grad), oracle.force(dims, U, chi, coeff=2.5, mode=0)) <= 1e-9


def test_solve_gradients_match_oracle(ctx):
    """L = Re(w^dag x), x = M^-1 b: grad_b = M^-1 w, grad_U from (x, M^-1 w)."""
    dims, mass = (4, 4, 6, 4), 0.3
    U = synth.gauge(dims, "haar", seed=85)
    b, w = _even(dims, 86), _even(dims, 87)
    Ut = dev(U).requires_grad_(True)
    bt = dev(b).requires_grad_(True)
    x = staggered_solve(Ut, bt, mass, ctx)
    L = (torch.conj(dev(w)) * x).sum().real
    L.backward()
    xo, _, _, _ = oracle.cg(dims, U, mass, b, tol=1e-13)
    lam, _, _, _ = oracle.cg(dims, U, mass, w, tol=1e-13)
    assert rel(host(x.detach()), xo) <= 1e-9
    assert rel(host(bt.grad), lam) <= 1e-9
    assert rel(host(Ut.grad), oracle.force(dims, U, xo, lam, mode=1)) <= 1e-9


def test_gradcheck_solve_and_action(ctx):
    """torch.autograd.gradcheck (fast mode) on 4^4 with unconstrained complex links."""
    dims = (4, 4, 4, 4)
    U = synth.gauge(dims, "haar", seed=88)
    Ut = dev(U).requires_grad_(True)
    bt = dev(_even(dims, 89)).requires_grad_(True)
    mask = dev(np.broadcast_to((np.indices((4, 4, 4, 4)).sum(0) % 2 == 0)[..., None], (4, 4, 4, 4, 3)).astype(np.complex128))

    def f_solve(u, b):
        return staggered_solve(u, b * mask, 0.3, ctx, tol=1e-13) * mask

    def f_action(u, b):
        return staggered_action(u, b * mask, 0.3, ctx, project=False, tol=1e-13)

    assert torch.autograd.gradcheck(f_solve, (Ut, bt), eps=1e-6, atol=1e-6, rtol=1e-5, fast_mode=True)
    assert torch.autograd.gradcheck(f_action, (Ut, bt), eps=1e-6, atol=1e-5, rtol=1e-5, fast_mode=True)


def test_autograd_functions_at_24x4_config(ctx):
    """The differentiation workload through both torch.autograd Functions: 24^4, smooth links
    eps = 0.3 (seed 1004), m = 0.05, phi from seed 2004 (and w from seed 2005 for the solve).

    StaggeredAction: S, grad_phi = 2 chi and the projected su(3) force.  StaggeredSolve with
    L = Re(w^dag x): x, grad_b = M^-1 w and the Euclidean link gradient.  The oracle's own CG
    (tol 1e-12) gives chi, x and lambda; the GPU's solves (tol 1e-12) may differ from them by
    kappa * 1e-12 each (kappa <= (m^2 + 64) / m^2), and quantities bilinear in them by twice
    that.  On the GPU's own vectors the gradients must equal the oracle's derivative formulas
    to 1e-12."""
    dims, mass, tol = (24, 24, 24, 24), 0.05, 1e-12
    kappa = (mass ** 2 + 64) / mass ** 2
    U = synth.gauge(dims, "smooth", seed=1004, eps=0.3)
    phi = _even(dims, 2004)
    w = _even(dims, 2005)

    print("24^4 action", flush=True)
    Ut = dev(U).requires_grad_(True)
    pt = dev(phi).requires_grad_(True)
    S = staggered_action(Ut, pt, mass, ctx, project=True, tol=tol)
    S.backward()
    chi_g = host(pt.grad) / 2.0      # grad_phi = 2 chi (the library scales by 2, exact)
    F = host(Ut.grad)
    chi_o, st, _, _ = oracle.cg(dims, U, mass, phi, tol=tol)
    assert st == 0
    assert rel(chi_g, chi_o) <= kappa * tol
    S_o = np.vdot(phi, chi_o).real
    assert abs(float(S) - S_o) <= 2 * kappa * tol * abs(S_o)
    assert rel(F, oracle.force(dims, U, chi_g)) <= 1e-12
    assert rel(F, oracle.force(dims, U, chi_o)) <= 2 * kappa * tol

    print("24^4 solve", flush=True)
    Ut2 = dev(U).requires_grad_(True)
    bt = dev(phi).requires_grad_(True)
    x = staggered_solve(Ut2, bt, mass, ctx, tol=tol)
    L = (torch.conj(dev(w)) * x).sum().real
    L.backward()
    x_g, lam_g, G = host(x.detach()), host(bt.grad), host(Ut2.grad)
    lam_o, st, _, _ = oracle.cg(dims, U, mass, w, tol=tol)
    assert st == 0
    assert rel(x_g, chi_o) <= kappa * tol
    assert rel(lam_g, lam_o) <= kappa * tol
    assert rel(G, oracle.force(dims, U, x_g, lam_g, mode=1)) <= 1e-12
    assert rel(G, oracle.force(dims, U, chi_o, lam_o, mode=1)) <= 2 * kappa * tol
