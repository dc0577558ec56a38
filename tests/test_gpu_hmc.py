"""HMC on the GPU against the oracle: plaquette action and force, kinetic energy,
link update, and whole trajectories (pure gauge, with the staggered pseudofermion,
mixed-precision solves, reversibility, the Metropolis decision)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import dev, host, rel

pytestmark = pytest.mark.gpu

lqs = pytest.importorskip("paper_2502_03249_amd")

RAGGED = (4, 6, 8, 10)


@pytest.fixture(scope="module")
def ctx():
    c = lqs.Context(0)
    yield c
    c.close()


def _eta(dims, seed):
    # complex Gaussian with density ~ exp(-|eta|^2): N(0, 1/2) parts
    return synth.source(dims, -1, seed=seed) / np.sqrt(2)


@pytest.mark.parametrize("dims,kind", [((4, 4, 4, 4), "haar"), (RAGGED, "smooth"), ((8, 8, 8, 16), "smooth")])
def test_gauge_action_force_kinetic(ctx, dims, kind):
    U = synth.gauge(dims, kind, seed=301, eps=0.5)
    Q = synth.momenta(dims, seed=302)
    beta = 5.7
    s = lqs.gauge_action(ctx, dims, dev(U), beta)
    want = oracle.plaquette_action(dims, U, beta)
    assert abs(s - want) <= 1e-12 * abs(want)
    F = host(lqs.gauge_force(ctx, dims, dev(U), beta, coeff=0.5))
    Fo = oracle.gauge_force(dims, U, beta, coeff=0.5)
    assert rel(F, Fo) <= 1e-13
    # accumulate mode: out += coeff F
    out = dev(Q)
    lqs.gauge_force(ctx, dims, dev(U), beta, coeff=-0.25, out=out, accumulate=True)
    assert rel(host(out), Q - 0.5 * Fo) <= 1e-13
    k = lqs.kinetic_energy(ctx, dims, dev(Q))
    assert abs(k - oracle.kinetic(dims, Q)) <= 1e-12 * oracle.kinetic(dims, Q)


@pytest.mark.parametrize("eps", [0.05, 0.7, 3.0])
def test_link_update(ctx, eps):
    dims = RAGGED
    U = synth.gauge(dims, "haar", seed=303)
    Q = synth.momenta(dims, seed=304)
    Ud = dev(U)
    lqs.link_update(ctx, dims, Ud, dev(Q), eps)
    got = host(Ud)
    assert rel(got, oracle.link_update(dims, U, Q, eps)) <= 1e-13
    # still SU(3)
    eye = np.eye(3)
    assert np.abs(got @ np.conj(np.swapaxes(got, -1, -2)) - eye).max() < 1e-13


def _run(ctx, dims, U, Q, pf, fermions, **kw):
    Ud, Qd = dev(U), dev(Q)
    prop = torch.empty_like(Ud)
    phi = torch.zeros((dims[3], dims[2], dims[1], dims[0], 3), dtype=torch.complex128, device=Ud.device)
    st = lqs.hmc_trajectory(ctx, dims, Ud, Qd, dev(pf) if pf is not None else None, fermions=fermions,
                            proposal=prop, phi_out=phi if fermions else None, **kw)
    return st, host(Ud), host(Qd), host(prop), host(phi)


@pytest.mark.parametrize("integ", ["leapfrog", "omelyan"])
def test_pure_gauge_trajectory(ctx, integ):
    dims = RAGGED
    U = synth.gauge(dims, "smooth", seed=305, eps=0.2)
    Q = synth.momenta(dims, seed=306)
    kw = dict(beta=5.5, tau=0.5, nsteps=6)
    st, U_ret, Q1, U1, _ = _run(ctx, dims, U, Q, None, 0, integrator=getattr(lqs, integ.upper()), **kw)
    o = oracle.hmc(dims, U, Q, None, 0.1, 5.5, 0.5, 6, integrator=integ, fermions=False)
    assert rel(U1, o["U1"]) <= 1e-12 and rel(Q1, o["Q1"]) <= 1e-12
    e = o["energies"]
    assert abs(st["k0"] - e[0]) <= 1e-12 * e[0] and abs(st["sg0"] - e[1]) <= 1e-12 * e[1]
    assert abs(st["k1"] - e[3]) <= 1e-12 * e[3] and abs(st["sg1"] - e[4]) <= 1e-12 * e[4]
    assert abs(st["dH"] - o["dH"]) <= 1e-12 * (e[0] + e[1])
    assert st["cg_solves"] == 0 and st["status"] == 0
    assert np.array_equal(U_ret, U1 if st["accepted"] else U)


@pytest.mark.parametrize("integ,n", [("leapfrog", 4), ("omelyan", 3)])
def test_trajectory_with_fermions_matches_oracle(ctx, integ, n):
    dims = RAGGED
    U = synth.gauge(dims, "smooth", seed=307, eps=0.2)
    Q = synth.momenta(dims, seed=308)
    eta = _eta(dims, 309)
    mass, beta, tau = 0.2, 5.5, 0.4
    st, U_ret, Q1, U1, phi = _run(ctx, dims, U, Q, eta, 1, beta=beta, mass=mass, tau=tau, nsteps=n,
                                  integrator=getattr(lqs, integ.upper()), tol=1e-13)
    o = oracle.hmc(dims, U, Q, eta, mass, beta, tau, n, integrator=integ, cg_tol=1e-13)
    assert st["status"] == 0 and o["status"] == 0
    assert rel(phi, o["phi"]) <= 1e-14
    # each solve meets ||phi - M chi|| <= 1e-13 ||phi||, so chi (and the fermion force, linear in
    # chi twice) is good to kappa * 1e-13 with kappa <= (m^2 + 64) / m^2 = 1601: about 3e-10
    bound = 2 * (mass ** 2 + 64) / mass ** 2 * 1e-13
    assert rel(U1, o["U1"]) <= bound and rel(Q1, o["Q1"]) <= bound
    e = o["energies"]
    for k, i in (("k0", 0), ("sg0", 1), ("sf0", 2), ("k1", 3), ("sg1", 4), ("sf1", 5)):
        assert abs(st[k] - e[i]) <= bound * abs(e[i]), k
    assert abs(st["dH"] - o["dH"]) <= bound * (e[0] + e[1] + e[2])
    # the start and end solves double as force solves: leapfrog n+1, Omelyan 2n+1 (merged boundaries)
    assert st["cg_solves"] == (n + 1 if integ == "leapfrog" else 2 * n + 1)
    assert st["accepted"] == o["accepted"]
    assert np.array_equal(U_ret, U1 if st["accepted"] else U)
    assert abs(st["plaquette"] - (1 - oracle.plaquette_action(dims, U_ret, 1.0) / (6 * np.prod(dims)))) < 1e-13


@pytest.mark.parametrize("inner,recon,tol", [(lqs.F32, 18, 1e-10), (lqs.F16, 12, 1e-10)])
def test_mixed_precision_solves_inside_trajectory(ctx, inner, recon, tol):
    dims = (8, 8, 8, 8)
    U = synth.gauge(dims, "smooth", seed=310, eps=0.2)
    Q = synth.momenta(dims, seed=311)
    eta = _eta(dims, 312)
    st, _, Q1, U1, _ = _run(ctx, dims, U, Q, eta, 1, beta=5.5, mass=0.1, tau=0.3, nsteps=3, tol=tol,
                            inner_prec=inner, inner_recon=recon, use_x0=True)
    o = oracle.hmc(dims, U, Q, eta, 0.1, 5.5, 0.3, 3, cg_tol=1e-13)
    assert st["status"] == 0
    # each solve is good to tol in the FP64 residual, so chi and the forces are good to
    # kappa * tol, kappa <= (m^2 + 64) / m^2 = 6401 at m = 0.1
    bound = 2 * (0.1 ** 2 + 64) / 0.1 ** 2 * tol
    assert rel(U1, o["U1"]) <= bound and rel(Q1, o["Q1"]) <= bound
    e = o["energies"]
    assert abs(st["dH"] - o["dH"]) <= bound * (e[0] + e[1] + e[2])


def test_reversibility_on_gpu(ctx):
    dims = RAGGED
    U = synth.gauge(dims, "smooth", seed=313, eps=0.2)
    Q = synth.momenta(dims, seed=314)
    eta = _eta(dims, 315)
    kw = dict(beta=5.5, mass=0.2, tau=0.4, nsteps=4, integrator=lqs.OMELYAN, tol=1e-14)
    st, _, Q1, U1, phi = _run(ctx, dims, U, Q, eta, 1, **kw)
    sb, _, Q2, U2, _ = _run(ctx, dims, U1, -Q1, phi, 2, **kw)
    assert st["status"] == 0 and sb["status"] == 0
    assert rel(U2, U) <= 1e-11 and rel(-Q2, Q) <= 1e-11
    assert abs(st["dH"] + sb["dH"]) <= 1e-8


def test_metropolis_and_rejection_keeps_links(ctx):
    dims = RAGGED
    U = synth.gauge(dims, "smooth", seed=316, eps=0.2)
    Q = synth.momenta(dims, seed=317)
    eta = _eta(dims, 318)
    kw = dict(beta=5.5, mass=0.2, tau=0.5, nsteps=2, tol=1e-12)
    st, _, _, _, _ = _run(ctx, dims, U, Q, eta, 1, **kw)
    assert st["dH"] > 0, "pick a trajectory with dH > 0"
    p = np.exp(-st["dH"])
    for u in (0.999 * p, min(1.001 * p, 0.999999)):
        s2, U_ret, _, U1, _ = _run(ctx, dims, U, Q, eta, 1, u=u, **kw)
        assert s2["accepted"] == (u < p)
        assert np.array_equal(U_ret, U1 if s2["accepted"] else U)


def test_invalid_arguments(ctx):
    dims = RAGGED
    U, Q = dev(synth.gauge(dims, "haar", seed=319)), dev(synth.momenta(dims, seed=320))
    for kw in (dict(nsteps=0), dict(tau=-1.0), dict(integrator=7), dict(u=1.0), dict(mass=0.0),
               dict(lam=0.6, integrator=lqs.OMELYAN)):
        args = dict(fermions=1, pf=dev(_eta(dims, 1)))
        args.update(kw)
        with pytest.raises(lqs.LqsError) as e:
            lqs.hmc_trajectory(ctx, dims, U, Q, **args)
        assert e.value.status == lqs.EINVAL
    # momenta aliasing the links
    with pytest.raises(lqs.LqsError) as e:
        lqs.hmc_trajectory(ctx, dims, U, U, pf=dev(_eta(dims, 1)), fermions=1)
    assert e.value.status == lqs.EINVAL


def test_force_tolerance_only_loosens_force_solves(ctx):
    """force_tol loosens the solves inside the trajectory; the S_f solves at both ends keep tol."""
    dims = (8, 8, 8, 8)
    U = synth.gauge(dims, "smooth", seed=321, eps=0.2)
    Q = synth.momenta(dims, seed=322)
    eta = _eta(dims, 323)
    kw = dict(beta=5.5, mass=0.1, tau=0.3, nsteps=4, integrator=lqs.OMELYAN, tol=1e-11, use_x0=True)
    tight, _, _, U1t, _ = _run(ctx, dims, U, Q, eta, 1, **kw)
    loose, _, _, U1l, _ = _run(ctx, dims, U, Q, eta, 1, force_tol=1e-6, **kw)
    assert tight["status"] == 0 and loose["status"] == 0
    assert loose["cg_solves"] == tight["cg_solves"] and loose["cg_iters"] < tight["cg_iters"]
    for k in ("k0", "sg0", "sf0"):
        assert abs(loose[k] - tight[k]) <= 1e-9 * abs(tight[k])
    # force errors of order kappa * 1e-6 move the end point slightly; S_f there is still exact
    o = oracle.hmc(dims, U1l, np.zeros_like(Q), None, 0.1, 5.5, 1e-9, 1, fermions=True,
                   phi=oracle.pseudofermion(dims, U, 0.1, eta), cg_tol=1e-12)
    assert abs(loose["sf1"] - o["energies"][2]) <= 1e-8 * abs(o["energies"][2])
    assert rel(U1l, U1t) <= 1e-4
