"""CPU FP64 oracle for the staggered even-odd solver -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps ``oracle.c`` (the operator, CG and fermion
derivative) and ``hmc.c`` (plaquette action and derivative, SU(3)
exponential, pseudofermion heat bath, one HMC trajectory) -- plain C, FP64,
OpenMP over sites in the operator, serial reductions -- through ctypes and
shares nothing with the GPU library.  Conventions and the definition of every
function are documented in the C sources.

Arrays are numpy complex128: links (4, Nt, Nz, Ny, Nx, 3, 3), colour-vector
fields (Nt, Nz, Ny, Nx, 3) on the full lattice, with zeros off the parity a
field lives on.  ``dims`` is (Nx, Ny, Nz, Nt).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "hmc.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build():
    cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
           "-o", _LIB + ".tmp"] + _SRCS + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    i32p = ctypes.POINTER(ctypes.c_int32)
    vp = ctypes.c_void_p
    d = ctypes.c_double
    i32 = ctypes.c_int32
    lib.ora_dslash.argtypes = [i32p, vp, vp, vp, i32]
    lib.ora_dslash.restype = None
    lib.ora_dslash_dagger.argtypes = [i32p, vp, vp, vp, i32]
    lib.ora_dslash_dagger.restype = None
    lib.ora_normal.argtypes = [i32p, vp, d, vp, vp]
    lib.ora_normal.restype = None
    lib.ora_true_residual.argtypes = [i32p, vp, d, vp, vp]
    lib.ora_true_residual.restype = d
    lib.ora_cg.argtypes = [i32p, vp, d, vp, vp, d, i32, i32p, ctypes.POINTER(d)]
    lib.ora_cg.restype = i32
    lib.ora_force.argtypes = [i32p, vp, vp, vp, d, i32, vp]
    lib.ora_force.restype = None
    lib.ora_threads.argtypes = []
    lib.ora_threads.restype = i32
    lib.ora_set_threads.argtypes = [i32]
    lib.ora_set_threads.restype = None
    lib.ora_expm3.argtypes = [vp, vp]
    lib.ora_expm3.restype = None
    lib.ora_plaquette_action.argtypes = [i32p, vp, d]
    lib.ora_plaquette_action.restype = d
    lib.ora_gauge_force.argtypes = [i32p, vp, d, d, vp]
    lib.ora_gauge_force.restype = None
    lib.ora_kinetic.argtypes = [i32p, vp]
    lib.ora_kinetic.restype = d
    lib.ora_pseudofermion.argtypes = [i32p, vp, d, vp, vp]
    lib.ora_pseudofermion.restype = None
    lib.ora_link_update.argtypes = [i32p, vp, vp, d]
    lib.ora_link_update.restype = None
    lib.ora_hmc.argtypes = [i32p, vp, vp, vp, d, d, d, i32, i32, d, i32, d, d, vp, vp, vp, i32p, i32p, i32p, vp]
    lib.ora_hmc.restype = i32
    _lib = lib
    return lib


def _dims(dims):
    d = np.ascontiguousarray(dims, dtype=np.int32)
    assert d.shape == (4,) and all(int(v) % 2 == 0 and v >= 2 for v in d), "extents must be even"
    return d, d.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _links(U, d):
    U = np.ascontiguousarray(U, dtype=np.complex128)
    assert U.shape == (4, d[3], d[2], d[1], d[0], 3, 3)
    return U


def _field(f, d):
    f = np.ascontiguousarray(f, dtype=np.complex128)
    assert f.shape == (d[3], d[2], d[1], d[0], 3)
    return f


def dslash(dims, U, x, out_parity=-1):
    """D x by eq. (1); out_parity 0/1 keeps only that output parity (the hop)."""
    d, dp = _dims(dims)
    U, x = _links(U, d), _field(x, d)
    out = np.empty_like(x)
    load().ora_dslash(dp, U.ctypes.data, x.ctypes.data, out.ctypes.data, int(out_parity))
    return out


def dslash_dagger(dims, U, x, out_parity=-1):
    """D^dag x, built as the conjugate transpose of the stencil (scatter form)."""
    d, dp = _dims(dims)
    U, x = _links(U, d), _field(x, d)
    out = np.empty_like(x)
    load().ora_dslash_dagger(dp, U.ctypes.data, x.ctypes.data, out.ctypes.data, int(out_parity))
    return out


def normal(dims, U, mass, x):
    """M x = m^2 x - D_eo D_oe x on even sites."""
    d, dp = _dims(dims)
    U, x = _links(U, d), _field(x, d)
    out = np.empty_like(x)
    load().ora_normal(dp, U.ctypes.data, float(mass), x.ctypes.data, out.ctypes.data)
    return out


def true_residual(dims, U, mass, b, x):
    """||b - M x|| / ||b|| over even sites."""
    d, dp = _dims(dims)
    U, b, x = _links(U, d), _field(b, d), _field(x, d)
    return load().ora_true_residual(dp, U.ctypes.data, float(mass), b.ctypes.data, x.ctypes.data)


def cg(dims, U, mass, b, tol=1e-10, max_iter=10000, x0=None):
    """Solve M x = b.  Returns (x, status, iterations, true relative residual)."""
    d, dp = _dims(dims)
    U, b = _links(U, d), _field(b, d)
    x = np.zeros_like(b) if x0 is None else _field(x0, d).copy()
    it = ctypes.c_int32(0)
    tr = ctypes.c_double(0.0)
    st = load().ora_cg(dp, U.ctypes.data, float(mass), b.ctypes.data, x.ctypes.data, float(tol),
                       int(max_iter), ctypes.byref(it), ctypes.byref(tr))
    return x, int(st), int(it.value), float(tr.value)


def force(dims, U, X, Y=None, coeff=1.0, mode=0):
    """Link derivative; mode 0: su(3) force F, mode 1: Euclidean gradient Pi^dag."""
    d, dp = _dims(dims)
    U, X = _links(U, d), _field(X, d)
    Yp = None
    if Y is not None:
        Y = _field(Y, d)
        Yp = Y.ctypes.data
    out = np.empty_like(U)
    load().ora_force(dp, U.ctypes.data, X.ctypes.data, Yp, float(coeff), int(mode), out.ctypes.data)
    return out


def threads():
    return int(load().ora_threads())


def set_threads(n):
    """Threads for the oracle's parallel regions."""
    load().ora_set_threads(int(n))


OMELYAN_LAMBDA = 0.1931833275037836


def expm3(A):
    """exp(A) of one 3x3 complex matrix (scaling and squaring of the Taylor series)."""
    A = np.ascontiguousarray(A, dtype=np.complex128)
    assert A.shape == (3, 3)
    out = np.empty_like(A)
    load().ora_expm3(A.ctypes.data, out.ctypes.data)
    return out


def plaquette_action(dims, U, beta):
    """S_g = beta sum_x sum_{mu<nu} (1 - Re tr P_{mu nu}(x) / 3)."""
    d, dp = _dims(dims)
    U = _links(U, d)
    return float(load().ora_plaquette_action(dp, U.ctypes.data, float(beta)))


def gauge_force(dims, U, beta, coeff=1.0):
    """coeff * F_g, F_g = (beta/3) TA(U V) with V the staple sum of each link."""
    d, dp = _dims(dims)
    U = _links(U, d)
    out = np.empty_like(U)
    load().ora_gauge_force(dp, U.ctypes.data, float(beta), float(coeff), out.ctypes.data)
    return out


def kinetic(dims, Q):
    """K = -sum_links tr(Q^2)."""
    d, dp = _dims(dims)
    Q = _links(Q, d)
    return float(load().ora_kinetic(dp, Q.ctypes.data))


def pseudofermion(dims, U, mass, eta):
    """phi = m eta_e - D_eo eta_o on even sites."""
    d, dp = _dims(dims)
    U, eta = _links(U, d), _field(eta, d)
    out = np.empty_like(eta)
    load().ora_pseudofermion(dp, U.ctypes.data, float(mass), eta.ctypes.data, out.ctypes.data)
    return out


def link_update(dims, U, Q, eps):
    """exp(eps Q) U on every link (returns a new array)."""
    d, dp = _dims(dims)
    U = _links(U, d).copy()
    Q = _links(Q, d)
    load().ora_link_update(dp, U.ctypes.data, Q.ctypes.data, float(eps))
    return U


def hmc(dims, U, Q, eta, mass, beta, tau, nsteps, integrator="leapfrog", lam=OMELYAN_LAMBDA, fermions=True,
        cg_tol=1e-12, u=0.5, phi=None):
    """One HMC trajectory.  The pseudofermion is made from the Gaussians eta on U, or given as phi
    (then eta is ignored).  Returns a dict with the proposal U1, Q1, the pseudofermion phi, the
    energies (K0, Sg0, Sf0, K1, Sg1, Sf1), dH, accepted, cg_iters, cg_solves, status."""
    d, dp = _dims(dims)
    U, Q = _links(U, d), _links(Q, d)
    zero = np.zeros((d[3], d[2], d[1], d[0], 3), np.complex128)
    mode = 0 if not fermions else (2 if phi is not None else 1)
    pf = _field(phi if phi is not None else (eta if eta is not None else zero), d)
    U1, Q1, phi_out = np.empty_like(U), np.empty_like(Q), np.empty_like(zero)
    en = np.zeros(6)
    acc, it, ns = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
    integ = {"leapfrog": 0, "omelyan": 1}[integrator]
    st = load().ora_hmc(dp, U.ctypes.data, Q.ctypes.data, pf.ctypes.data, float(mass), float(beta), float(tau),
                        int(nsteps), integ, float(lam), mode, float(cg_tol), float(u), U1.ctypes.data,
                        Q1.ctypes.data, en.ctypes.data, ctypes.byref(acc), ctypes.byref(it), ctypes.byref(ns),
                        phi_out.ctypes.data)
    dh = (en[3] + en[4] + en[5]) - (en[0] + en[1] + en[2])
    return {"U1": U1, "Q1": Q1, "phi": phi_out, "energies": en, "dH": float(dh), "accepted": bool(acc.value),
            "cg_iters": int(it.value), "cg_solves": int(ns.value), "status": int(st)}
