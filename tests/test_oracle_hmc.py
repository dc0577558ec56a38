"""Pins of the HMC part of the oracle (plaquette action and derivative, SU(3)
exponential, momenta, heat bath, trajectory) against closed forms, library
routines, finite differences and the invariants of Hamiltonian dynamics."""
import numpy as np
import pytest
import scipy.linalg

import oracle
import synth
from latt import gauge_transform, on_parity, rel, su3_generators

DIMS = (4, 4, 4, 4)


def test_expm3_matches_scipy():
    rng = np.random.default_rng(7)
    for scale in (1e-3, 0.3, 1.0, 4.0, 30.0):
        A = scale * (rng.normal(size=(3, 3)) + 1j * rng.normal(size=(3, 3)))
        assert rel(oracle.expm3(A), scipy.linalg.expm(A)) < 1e-13
    # an anti-Hermitian traceless argument gives an SU(3) matrix
    Q = synth.momenta(DIMS, seed=1)[0, 0, 0, 0, 0]
    E = oracle.expm3(0.7 * Q)
    assert np.abs(E @ E.conj().T - np.eye(3)).max() < 1e-14
    assert abs(np.linalg.det(E) - 1) < 1e-14


def test_plaquette_action_unit_and_abelian_flux():
    nx, ny, nz, nt = 4, 6, 4, 4
    dims = (nx, ny, nz, nt)
    U = np.zeros((4, nt, nz, ny, nx, 3, 3), np.complex128)
    U[...] = np.eye(3)
    assert oracle.plaquette_action(dims, U, 5.5) == 0.0
    # U_x(x) = diag(e^{i phi y}, e^{-i phi y}, 1) with phi = 2 pi k / Ny: every (x, y) plaquette
    # is diag(e^{-i phi}, e^{i phi}, 1), every other plaquette is 1
    phi = 2 * np.pi * 2 / ny
    y = np.arange(ny)
    U[0, :, :, :, :, 0, 0] = np.exp(1j * phi * y)[None, None, :, None]
    U[0, :, :, :, :, 1, 1] = np.exp(-1j * phi * y)[None, None, :, None]
    vol = nx * ny * nz * nt
    want = 5.5 * vol * (1 - (2 * np.cos(phi) + 1) / 3)
    assert abs(oracle.plaquette_action(dims, U, 5.5) - want) < 1e-12 * want


def test_plaquette_action_gauge_invariant_and_linear_in_beta():
    U = synth.gauge(DIMS, "haar", seed=201)
    G = synth.site_haar(DIMS, seed=202)
    s = oracle.plaquette_action(DIMS, U, 1.0)
    assert abs(oracle.plaquette_action(DIMS, gauge_transform(U, G), 1.0) - s) < 1e-12 * abs(s)
    assert abs(oracle.plaquette_action(DIMS, U, 6.0) - 6.0 * s) < 1e-12 * abs(s)
    # Haar links: <Re tr P> = 0, so S / (beta * 6 V) is close to 1
    assert abs(s / (6 * 256) - 1) < 0.05


def test_gauge_force_matches_finite_differences():
    U = synth.gauge(DIMS, "smooth", seed=203, eps=0.6)
    beta = 5.7
    F = oracle.gauge_force(DIMS, U, beta)
    # su(3): anti-Hermitian and traceless
    assert np.abs(F + np.conj(np.swapaxes(F, -1, -2))).max() < 1e-14
    assert np.abs(np.trace(F, axis1=-2, axis2=-1)).max() < 1e-14
    T = su3_generators()  # i lambda_a / 2: anti-Hermitian, tr(T_a T_b) = -delta_ab / 2
    rng = np.random.default_rng(5)
    h = 1e-5
    worst = 0.0
    for _ in range(6):
        mu = int(rng.integers(4))
        site = tuple(int(rng.integers(n)) for n in (DIMS[3], DIMS[2], DIMS[1], DIMS[0]))
        for a in range(8):
            vals = []
            for sgn in (1, -1):
                V = U.copy()
                V[(mu,) + site] = scipy.linalg.expm(sgn * h * T[a]) @ U[(mu,) + site]
                vals.append(oracle.plaquette_action(DIMS, V, beta))
            fd = (vals[0] - vals[1]) / (2 * h)
            an = np.real(np.trace(F[(mu,) + site].conj().T @ T[a]))
            worst = max(worst, abs(fd - an) / (abs(an) + 1e-3))
    assert worst < 1e-6


def test_gauge_force_coefficient():
    U = synth.gauge(DIMS, "haar", seed=204)
    assert rel(oracle.gauge_force(DIMS, U, 5.0, coeff=-0.25), -0.25 * oracle.gauge_force(DIMS, U, 5.0)) < 1e-15


def test_momenta_and_kinetic_energy():
    Q = synth.momenta(DIMS, seed=205)
    T = su3_generators()
    # coefficients q_a = -2 tr(Q T_a); Q is rebuilt from them exactly
    q = np.stack([-2 * np.einsum("...ij,ji->...", Q, Ta) for Ta in T], axis=-1)
    assert np.abs(q.imag).max() < 1e-14
    assert rel(np.einsum("...a,aij->...ij", q.real, np.stack(T)), Q) < 1e-14
    assert abs(oracle.kinetic(DIMS, Q) - 0.5 * np.sum(q.real ** 2)) < 1e-11 * oracle.kinetic(DIMS, Q)
    # heat bath: q_a ~ N(0,1) -> <K> = 4 per link
    assert abs(oracle.kinetic(DIMS, Q) / (4 * 256) - 4) < 0.2


def test_pseudofermion_heat_bath():
    """phi = m eta_e - D_eo eta_o; with eta = (m zeta, D_oe zeta) it is M zeta, so phi^dag M^-1 phi = |eta|^2."""
    U = synth.gauge(DIMS, "haar", seed=206)
    mass = 0.3
    zeta = synth.source(DIMS, 0, seed=207)
    eta = mass * zeta + oracle.dslash(DIMS, U, zeta, 1)
    phi = oracle.pseudofermion(DIMS, U, mass, eta)
    assert rel(phi, oracle.normal(DIMS, U, mass, zeta)) < 1e-14
    x, st, _, _ = oracle.cg(DIMS, U, mass, phi, tol=1e-13)
    assert st == 0
    sf = np.vdot(phi, x).real
    assert abs(sf - np.vdot(eta, eta).real) < 1e-10 * sf
    # odd-site output stays zero
    assert np.abs(on_parity(phi, DIMS, 1)).max() == 0.0


def test_link_update_matches_scipy():
    U = synth.gauge(DIMS, "haar", seed=208)
    Q = synth.momenta(DIMS, seed=209)
    U1 = oracle.link_update(DIMS, U, Q, 0.13)
    idx = [(0, 0, 0, 0, 0), (1, 1, 2, 3, 0), (3, 3, 3, 3, 3), (2, 0, 1, 0, 3)]
    for i in idx:
        assert rel(U1[i], scipy.linalg.expm(0.13 * Q[i]) @ U[i]) < 1e-14


def test_free_molecular_dynamics():
    """beta = 0, no fermions: Q is constant and U(tau) = exp(tau Q) U for both integrators."""
    U = synth.gauge(DIMS, "haar", seed=210)
    Q = synth.momenta(DIMS, seed=211)
    for integ in ("leapfrog", "omelyan"):
        r = oracle.hmc(DIMS, U, Q, None, 0.1, 0.0, 0.8, 7, integrator=integ, fermions=False)
        assert np.array_equal(r["Q1"], Q)
        for i in [(0, 0, 0, 0, 0), (3, 1, 2, 3, 1)]:
            assert rel(r["U1"][i], scipy.linalg.expm(0.8 * Q[i]) @ U[i]) < 1e-13
        assert abs(r["dH"]) < 1e-9


def _dh(nsteps, integ, fermions, beta=5.5, seed=212):
    U = synth.gauge(DIMS, "smooth", seed=seed, eps=0.2)
    Q = synth.momenta(DIMS, seed=seed + 1)
    eta = synth.source(DIMS, -1, seed=seed + 2) / np.sqrt(2)
    return oracle.hmc(DIMS, U, Q, eta, 0.2, beta, 0.5, nsteps, integrator=integ, fermions=fermions)


@pytest.mark.parametrize("beta,fermions,n", [(5.5, False, 8), (5.5, True, 8), (0.0, True, 16)])
@pytest.mark.parametrize("integ", ["leapfrog", "omelyan"])
def test_energy_violation_is_second_order(integ, beta, fermions, n):
    """Both integrators are second order: halving the step divides dH by about 4 (gauge and
    fermion forces together, and the fermion force alone).  A wrong sign or factor in either
    force would leave a dH that does not shrink with the step."""
    a, b = _dh(n, integ, fermions, beta), _dh(2 * n, integ, fermions, beta)
    assert a["status"] == 0 and b["status"] == 0
    ratio = a["dH"] / b["dH"]
    assert 3.6 < ratio < 4.4
    if fermions:
        assert a["cg_solves"] == (n + 1 + 2 if integ == "leapfrog" else 3 * n + 2)


def test_omelyan_beats_leapfrog_at_equal_step():
    assert abs(_dh(10, "omelyan", True)["dH"]) < abs(_dh(10, "leapfrog", True)["dH"])


def test_reversibility():
    """Running the proposal backwards (negated momenta, same pseudofermion) returns to the start."""
    U = synth.gauge(DIMS, "smooth", seed=220, eps=0.4)
    Q = synth.momenta(DIMS, seed=221)
    eta = synth.source(DIMS, -1, seed=222) / np.sqrt(2)
    for integ in ("leapfrog", "omelyan"):
        f = oracle.hmc(DIMS, U, Q, eta, 0.2, 5.5, 0.5, 6, integrator=integ, cg_tol=1e-14)
        b = oracle.hmc(DIMS, f["U1"], -f["Q1"], None, 0.2, 5.5, 0.5, 6, integrator=integ, cg_tol=1e-14,
                       phi=f["phi"])
        assert f["status"] == 0 and b["status"] == 0
        assert rel(b["U1"], U) < 1e-10 and rel(-b["Q1"], Q) < 1e-10
        assert abs(b["dH"] + f["dH"]) < 1e-9
        # pure gauge: exact to rounding
        g = oracle.hmc(DIMS, U, Q, None, 0.2, 5.5, 0.5, 6, integrator=integ, fermions=False)
        gb = oracle.hmc(DIMS, g["U1"], -g["Q1"], None, 0.2, 5.5, 0.5, 6, integrator=integ, fermions=False)
        assert rel(gb["U1"], U) < 1e-13 and rel(-gb["Q1"], Q) < 1e-13


def test_metropolis_decision():
    U = synth.gauge(DIMS, "smooth", seed=212, eps=0.2)
    Q = synth.momenta(DIMS, seed=213)
    eta = synth.source(DIMS, -1, seed=214) / np.sqrt(2)
    r = oracle.hmc(DIMS, U, Q, eta, 0.2, 5.5, 0.5, 8, integrator="omelyan")
    p = np.exp(-r["dH"])
    assert 0.0 < p < 1.0, "pick a trajectory with dH > 0 so both outcomes occur"
    for u in (0.999 * p, 1.001 * p):
        s = oracle.hmc(DIMS, U, Q, eta, 0.2, 5.5, 0.5, 8, integrator="omelyan", u=u)
        assert s["dH"] == r["dH"]
        assert s["accepted"] == (u < p)
