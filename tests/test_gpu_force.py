"""GPU link derivative against the oracle and against finite differences."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, field, gauge, host, lex_of, rel
from latt import expm_su3, su3_generators

pytestmark = pytest.mark.gpu

lqs = pytest.importorskip("paper_2502_03249_amd")


@pytest.fixture(scope="module")
def ctx():
    c = lqs.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (4, 6, 8, 10)])
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("same", [True, False])
def test_force_matches_oracle(ctx, dims, mode, same):
    U = synth.gauge(dims, "haar", seed=71)
    X = synth.source(dims, 0, seed=72)
    Y = synth.source(dims, 0, seed=73)
    g = gauge(ctx, dims, U)
    Xf = field(ctx, dims, X, 0)
    Yf = None if same else field(ctx, dims, Y, 0)
    got = host(lqs.fermion_force(ctx, g, Xf, Yf, coeff=0.75, mode=mode))
    want = oracle.force(dims, U, X, None if same else Y, coeff=0.75, mode=mode)
    assert rel(got, want) <= 1e-13


def _gpu_solve(ctx, dims, U, mass, phi, tol=1e-12):
    g = gauge(ctx, dims, U)
    bf = field(ctx, dims, phi, 0)
    xf = bf.like().zero_()
    st = lqs.cg_solve(ctx, [(g, mass, bf, xf)], tol=tol)
    assert st[0]["status"] == 0
    return g, xf


def test_force_24x4_config_fd_and_oracle(ctx):
    """24^4, smooth links eps = 0.3 (seed 1004), m = 0.05, source seed 2004; FD links from seed 3004.

    The GPU force on the GPU's chi matches the oracle force on the same chi,
    and central differences (h = 1e-4) of S = phi^dag M^-1 phi along
    U -> exp(+-h A) U, through S(U+) - S(U-) = chi+^dag (M- - M+) chi-, match
    Re tr(F^dag A) on 8 links x 8 generators.
    """
    dims, mass = (24, 24, 24, 24), 0.05
    U = synth.gauge(dims, "smooth", seed=1004, eps=0.3)
    phi = synth.source(dims, 0, seed=2004)
    g, chif = _gpu_solve(ctx, dims, U, mass, phi)
    chi = lex_of(ctx, chif)
    F = host(lqs.fermion_force(ctx, g, chif))
    Fo = oracle.force(dims, U, chi)
    assert rel(F, Fo) <= 1e-12
    rng = np.random.default_rng(3004)
    gens = su3_generators()
    h = 1e-4
    worst = 0.0
    for _ in range(8):
        link = (int(rng.integers(4)),) + tuple(int(rng.integers(n)) for n in dims[::-1])
        for A in gens:
            Up, Um = U.copy(), U.copy()
            Up[link] = expm_su3(h * A) @ U[link]
            Um[link] = expm_su3(-h * A) @ U[link]
            _, cpf = _gpu_solve(ctx, dims, Up, mass, phi)
            _, cmf = _gpu_solve(ctx, dims, Um, mass, phi)
            cp, cm = lex_of(ctx, cpf), lex_of(ctx, cmf)
            ds = np.vdot(cp, oracle.normal(dims, Um, mass, cm) - oracle.normal(dims, Up, mass, cm)).real
            an = np.trace(np.conj(F[link]).T @ A).real
            worst = max(worst, abs(ds / (2 * h) - an) / max(abs(an), 1e-3))
    assert worst <= 1e-6, worst
