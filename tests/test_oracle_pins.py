"""Pins of the CPU oracle against facts the mathematics fixes (no GPU).

Each test ties one oracle function to a closed form, an invariant, a brute-
force computation or a finite difference, chosen so that a dropped term, a
wrong sign, a wrong neighbour or link index, a transposed link or a missing
boundary sign fails at least one of them.
"""
import numpy as np
import pytest

import oracle
import synth
from latt import (apply_site, free_momenta, gauge_transform, on_parity, parity_mask, plane_wave, rel, shift,
                  su3_generators, expm_su3)

SMALL = (4, 4, 4, 4)
ASYM = (4, 6, 8, 10)


def _rand_field(dims, seed):
    rng = np.random.default_rng(seed)
    nx, ny, nz, nt = dims
    return rng.normal(size=(nt, nz, ny, nx, 3)) + 1j * rng.normal(size=(nt, nz, ny, nx, 3))


# --- Dslash, free field -------------------------------------------------------------

@pytest.mark.parametrize("dims", [SMALL, ASYM, (2, 4, 2, 6)])
def test_free_field_two_hop_closed_form(dims):
    """U = 1: D^2 phi(x) = sum_mu [s phi(x+2mu) - 2 phi(x) + s phi(x-2mu)], s = -1 across the t boundary.

    Cross terms cancel because eta_mu(x) eta_nu(x+nu) = -eta_nu(x) eta_mu(x+mu) for mu != nu;
    a wrong phase convention or a missing boundary sign breaks the identity.
    """
    U = synth.gauge(dims, "identity")
    phi = _rand_field(dims, 1)
    d2 = oracle.dslash(dims, U, oracle.dslash(dims, U, phi))
    nt = dims[3]
    t = np.arange(nt)[:, None, None, None, None]
    expect = -8.0 * phi
    for mu in range(4):
        fwd, bwd = shift(phi, mu, 2), shift(phi, mu, -2)
        if mu == 3:
            fwd = fwd * np.where(t >= nt - 2, -1.0, 1.0)
            bwd = bwd * np.where(t <= 1, -1.0, 1.0)
        expect = expect + fwd + bwd
    assert rel(d2, expect) < 1e-14


def _dense(dims, U, fn):
    nx, ny, nz, nt = dims
    n = nx * ny * nz * nt * 3
    cols = []
    for k in range(n):
        e = np.zeros(n, np.complex128)
        e[k] = 1.0
        cols.append(fn(dims, U, e.reshape(nt, nz, ny, nx, 3)).reshape(-1))
    return np.stack(cols, axis=1)


def test_free_field_spectrum():
    """Eigenvalues of D/2 on 4^4 with U = 1 are +-i sqrt(sum_mu sin^2 p_mu) (antiperiodic p_t)."""
    U = synth.gauge(SMALL, "identity")
    D = _dense(SMALL, U, oracle.dslash)
    assert np.abs(D + D.conj().T).max() < 1e-14
    ev = np.linalg.eigvalsh(1j * D / 2)          # iD/2 is Hermitian
    mag = np.sort(np.abs(ev))
    p = free_momenta(SMALL)
    expect = np.sort(np.repeat(np.sqrt((np.sin(p) ** 2).sum(axis=1)), 3))
    assert np.abs(mag - expect).max() < 1e-12
    assert np.abs(np.sort(ev) + np.sort(ev)[::-1]).max() < 1e-12  # +- pairs


@pytest.mark.parametrize("n", [(0, 0, 0, 0), (1, 2, 3, 1), (3, 1, 0, 2)])
def test_free_field_plane_wave_normal_op(n):
    """M f_e = (m^2 + 4 sum_mu sin^2 p_mu) f_e for a plane wave f_e on the even sites."""
    dims, mass = (4, 4, 6, 8), 0.3
    U = synth.gauge(dims, "identity")
    f, p = plane_wave(dims, n, [1.0, 0.5 - 0.25j, -0.75j])
    fe = on_parity(f, dims, 0)
    lam = mass ** 2 + 4 * sum(np.sin(q) ** 2 for q in p)
    assert rel(oracle.normal(dims, U, mass, fe), lam * fe) < 1e-14


# --- Dslash, any gauge field --------------------------------------------------------

@pytest.mark.parametrize("dims", [SMALL, ASYM])
def test_anti_hermiticity(dims):
    """<x, D y> = -<D x, y>, and the stencil's conjugate transpose equals -D."""
    U = synth.gauge(dims, "haar", seed=7)
    x, y = _rand_field(dims, 2), _rand_field(dims, 3)
    lhs = np.vdot(x, oracle.dslash(dims, U, y))
    rhs = -np.vdot(oracle.dslash(dims, U, x), y)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    dy = oracle.dslash(dims, U, y)
    assert rel(oracle.dslash_dagger(dims, U, y), -dy) < 1e-14
    for p in (0, 1):
        assert rel(oracle.dslash_dagger(dims, U, y, p), -oracle.dslash(dims, U, y, p)) < 1e-14


@pytest.mark.parametrize("dims", [SMALL, ASYM])
def test_eps_hermiticity_and_parity_blocks(dims):
    """eps D eps = -D with eps(x) = (-1)^(x+y+z+t); D maps each parity to the other."""
    U = synth.gauge(dims, "haar", seed=8)
    phi = _rand_field(dims, 4)
    eps = np.where(parity_mask(dims, 0), 1.0, -1.0)[..., None]
    assert rel(eps * oracle.dslash(dims, U, eps * phi), -oracle.dslash(dims, U, phi)) < 1e-14
    even = on_parity(phi, dims, 0)
    out = oracle.dslash(dims, U, even)
    assert np.abs(on_parity(out, dims, 0)).max() == 0.0
    assert rel(oracle.dslash(dims, U, even, 1), out) == 0.0


@pytest.mark.parametrize("dims", [SMALL, ASYM])
def test_gauge_covariance(dims):
    """D[U^G](G phi) = G D[U] phi for a Haar gauge transformation G."""
    U = synth.gauge(dims, "haar", seed=9)
    G = synth.site_haar(dims, seed=10)
    phi = _rand_field(dims, 5)
    lhs = oracle.dslash(dims, gauge_transform(U, G), apply_site(G, phi))
    rhs = apply_site(G, oracle.dslash(dims, U, phi))
    assert rel(lhs, rhs) < 1e-13


def test_pure_gauge_closed_form():
    """U_{x,mu} = G_x G^dag_{x+mu} gives D = G D_free G^dag; D_free is pinned above."""
    dims = ASYM
    G = synth.site_haar(dims, seed=11)
    U = gauge_transform(synth.gauge(dims, "identity"), G)
    phi = _rand_field(dims, 6)
    lhs = oracle.dslash(dims, U, phi)
    Gdag = np.conj(np.swapaxes(G, -1, -2))
    rhs = apply_site(G, oracle.dslash(dims, synth.gauge(dims, "identity"), apply_site(Gdag, phi)))
    assert rel(lhs, rhs) < 1e-13


def test_dense_spectrum_random_links():
    """Brute force on 4^4 Haar links: D is anti-Hermitian, eigenvalues purely imaginary in +- pairs."""
    U = synth.gauge(SMALL, "haar", seed=12)
    D = _dense(SMALL, U, oracle.dslash)
    assert np.abs(D + D.conj().T).max() < 1e-14
    ev = np.linalg.eigvals(D)
    assert np.abs(ev.real).max() < 1e-12
    im = np.sort(ev.imag)
    assert np.abs(im + im[::-1]).max() < 1e-11


# --- Normal operator and CG ---------------------------------------------------------

def _dense_even(dims, U, mass):
    mask = parity_mask(dims, 0).reshape(-1)
    idx = np.nonzero(np.repeat(mask, 3))[0]
    nx, ny, nz, nt = dims
    cols = []
    for k in idx:
        e = np.zeros(nx * ny * nz * nt * 3, np.complex128)
        e[k] = 1.0
        cols.append(oracle.normal(dims, U, mass, e.reshape(nt, nz, ny, nx, 3)).reshape(-1)[idx])
    return np.stack(cols, axis=1), idx


def test_normal_operator_from_dense_dslash():
    """Dense M equals m^2 - D_eo D_oe assembled from the dense D; M is HPD with lambda_min >= m^2."""
    mass = 0.1
    U = synth.gauge(SMALL, "haar", seed=1000)
    M, idx = _dense_even(SMALL, U, mass)
    D = _dense(SMALL, U, oracle.dslash)
    mask = np.repeat(parity_mask(SMALL, 0).reshape(-1), 3)
    odd = np.nonzero(~mask)[0]
    D_eo = D[np.ix_(idx, odd)]
    D_oe = D[np.ix_(odd, idx)]
    assert np.abs(M - (mass ** 2 * np.eye(len(idx)) - D_eo @ D_oe)).max() < 1e-13
    assert np.abs(M - M.conj().T).max() < 1e-13
    lam = np.linalg.eigvalsh(M)
    assert lam.min() >= mass ** 2 * (1 - 1e-10)


def test_cg_matches_dense_solve():
    """Configuration 4^4, Haar links (seed 1000), Gaussian even source (seed 2000), m = 0.1."""
    mass = 0.1
    U = synth.gauge(SMALL, "haar", seed=1000)
    b = synth.source(SMALL, 0, seed=2000)
    x, st, it, tr = oracle.cg(SMALL, U, mass, b, tol=1e-10)
    assert st == 0 and tr <= 1e-10
    M, idx = _dense_even(SMALL, U, mass)
    xd = np.linalg.solve(M, b.reshape(-1)[idx])
    kappa = np.linalg.cond(M)
    assert rel(x.reshape(-1)[idx], xd) <= kappa * 1e-10
    assert np.abs(on_parity(x, SMALL, 1)).max() == 0.0


def test_true_residual_from_dense_operator():
    """||b - M x|| / ||b|| on even fields equals the same norm formed with the dense M (itself
    pinned to the dense D above), for an arbitrary x, and vanishes to rounding at the dense solution."""
    mass = 0.1
    U = synth.gauge(SMALL, "haar", seed=1000)
    b = synth.source(SMALL, 0, seed=2000)
    x = on_parity(_rand_field(SMALL, 7), SMALL, 0)
    M, idx = _dense_even(SMALL, U, mass)
    be, xe = b.reshape(-1)[idx], x.reshape(-1)[idx]
    want = np.linalg.norm(be - M @ xe) / np.linalg.norm(be)
    assert abs(oracle.true_residual(SMALL, U, mass, b, x) - want) <= 1e-12 * want
    xs = np.zeros(b.size, np.complex128)
    xs[idx] = np.linalg.solve(M, be)
    assert oracle.true_residual(SMALL, U, mass, b, xs.reshape(b.shape)) <= 1e-13


def test_cg_plane_wave_exact_solution():
    """Free field: the solution for a plane-wave source is f_e / (m^2 + 4 sum sin^2 p)."""
    dims, mass = (8, 8, 8, 8), 0.05
    U = synth.gauge(dims, "identity")
    f, p = plane_wave(dims, (1, 3, 2, 0), [0.3, -1.0j, 0.7])
    fe = on_parity(f, dims, 0)
    lam = mass ** 2 + 4 * sum(np.sin(q) ** 2 for q in p)
    x, st, it, tr = oracle.cg(dims, U, mass, fe, tol=1e-12)
    assert st == 0
    assert rel(x, fe / lam) < 1e-11


def test_cg_warm_start_and_limits():
    """Resume from a partial solve reaches the same x; max_iter exhaustion reports status 1."""
    mass = 0.1
    U = synth.gauge(SMALL, "haar", seed=1000)
    b = synth.source(SMALL, 0, seed=2000)
    x_full, st, _, _ = oracle.cg(SMALL, U, mass, b, tol=1e-10)
    x_part, st1, _, tr1 = oracle.cg(SMALL, U, mass, b, tol=1e-5)
    assert st1 == 0 and tr1 <= 1e-5
    x_res, st2, _, tr2 = oracle.cg(SMALL, U, mass, b, tol=1e-10, x0=x_part)
    assert st2 == 0 and tr2 <= 1e-10
    assert rel(x_res, x_full) < 1e-7
    _, st3, it3, _ = oracle.cg(SMALL, U, mass, b, tol=1e-10, max_iter=5)
    assert st3 == 1 and it3 == 5


# --- Force (link derivative) ---------------------------------------------------------

def _solve(dims, U, mass, b):
    x, st, _, _ = oracle.cg(dims, U, mass, b, tol=1e-13, max_iter=20000)
    assert st == 0
    return x


def _links_to_check(dims, n, seed):
    rng = np.random.default_rng(seed)
    nx, ny, nz, nt = dims
    return [(int(rng.integers(4)), int(rng.integers(nt)), int(rng.integers(nz)), int(rng.integers(ny)),
             int(rng.integers(nx))) for _ in range(n)]


def test_force_finite_differences():
    """dS/dw along U -> exp(w A) U equals Re tr(F^dag A); S = phi^dag M^-1 phi.

    Central differences with h = 1e-4 through S(U+) - S(U-) = chi+^dag (M- - M+) chi-,
    8 links (both parities) x 8 generators.
    """
    dims, mass = SMALL, 0.2
    U = synth.gauge(dims, "smooth", seed=1004, eps=0.3)
    phi = synth.source(dims, 0, seed=2004)
    chi = _solve(dims, U, mass, phi)
    F = oracle.force(dims, U, chi)
    gens = su3_generators()
    h = 1e-4
    worst = 0.0
    for link in _links_to_check(dims, 8, 3004):
        for A in gens:
            Up, Um = U.copy(), U.copy()
            Up[link] = expm_su3(h * A) @ U[link]
            Um[link] = expm_su3(-h * A) @ U[link]
            cp, cm = _solve(dims, Up, mass, phi), _solve(dims, Um, mass, phi)
            ds = np.vdot(cp, oracle.normal(dims, Um, mass, cm) - oracle.normal(dims, Up, mass, cm)).real
            fd = ds / (2 * h)
            an = np.trace(np.conj(F[link]).T @ A).real
            worst = max(worst, abs(fd - an) / max(abs(an), 1e-3))
    assert worst < 1e-6
    # F is traceless anti-Hermitian.
    assert np.abs(F + np.conj(np.swapaxes(F, -1, -2))).max() < 1e-12
    assert np.abs(np.trace(F, axis1=-2, axis2=-1)).max() < 1e-12


def test_force_euclidean_gradient_general_loss():
    """Mode 1 gives dL/dRe U + i dL/dIm U for L = Re(w^dag M^-1 phi), with X = chi, Y = M^-1 w.

    Unconstrained entry perturbations (U leaves SU(3)); the loss is exact in the FD up to O(h^2).
    """
    dims, mass = SMALL, 0.3
    U = synth.gauge(dims, "haar", seed=21)
    phi = synth.source(dims, 0, seed=22)
    w = synth.source(dims, 0, seed=23)
    chi = _solve(dims, U, mass, phi)
    lam = _solve(dims, U, mass, w)
    G = oracle.force(dims, U, chi, lam, coeff=1.0, mode=1)
    h = 1e-5
    worst = 0.0
    for link in _links_to_check(dims, 6, 24):
        for (a, b) in [(0, 0), (1, 2), (2, 0)]:
            for unit in (1.0, 1j):
                Up, Um = U.copy(), U.copy()
                Up[link + (a, b)] += h * unit
                Um[link + (a, b)] -= h * unit
                lp = np.vdot(w, _solve(dims, Up, mass, phi)).real
                lm = np.vdot(w, _solve(dims, Um, mass, phi)).real
                fd = (lp - lm) / (2 * h)
                an = G[link + (a, b)].real if unit == 1.0 else G[link + (a, b)].imag
                worst = max(worst, abs(fd - an) / max(abs(an), 1e-3))
    assert worst < 1e-5


def test_force_symmetric_in_x_y_and_action_form():
    """Pi(X, Y) = Pi(Y, X); with X = Y = chi the projected force is -TA(U Pi)."""
    dims, mass = ASYM, 0.2
    U = synth.gauge(dims, "haar", seed=31)
    X, Y = synth.source(dims, 0, seed=32), synth.source(dims, 0, seed=33)
    g1 = oracle.force(dims, U, X, Y, mode=1)
    g2 = oracle.force(dims, U, Y, X, mode=1)
    assert rel(g1, g2) < 1e-14
    gx = oracle.force(dims, U, X, None, mode=1)
    F = oracle.force(dims, U, X, None, mode=0)
    upi = U @ np.conj(np.swapaxes(gx, -1, -2))
    ah = 0.5 * (upi - np.conj(np.swapaxes(upi, -1, -2)))
    ta = ah - np.trace(ah, axis1=-2, axis2=-1)[..., None, None] / 3 * np.eye(3)
    assert rel(F, -ta) < 1e-14


def test_force_gauge_covariance():
    """F[U^G, G X] = G F[U, X] G^dag link by link."""
    dims = SMALL
    U = synth.gauge(dims, "haar", seed=41)
    G = synth.site_haar(dims, seed=42)
    X = synth.source(dims, 0, seed=43)
    F = oracle.force(dims, U, X)
    FG = oracle.force(dims, gauge_transform(U, G), apply_site(G, X))
    Gdag = np.conj(np.swapaxes(G, -1, -2))
    assert rel(FG, G[None] @ F @ Gdag[None]) < 1e-13


def test_grad_phi_exact():
    """S is quadratic in phi: central FD of S along delta equals Re((2 chi)^dag delta) exactly."""
    dims, mass = SMALL, 0.2
    U = synth.gauge(dims, "haar", seed=51)
    phi = synth.source(dims, 0, seed=52)
    delta = synth.source(dims, 0, seed=53)
    chi = _solve(dims, U, mass, phi)
    h = 0.5
    sp = np.vdot(phi + h * delta, _solve(dims, U, mass, phi + h * delta)).real
    sm = np.vdot(phi - h * delta, _solve(dims, U, mass, phi - h * delta)).real
    assert abs((sp - sm) / (2 * h) - np.vdot(2 * chi, delta).real) < 1e-9 * abs(sp)
