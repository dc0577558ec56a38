"""Seeded synthetic inputs (gauge fields, gauge transformations, sources).

Shared by the CPU oracle tests, the GPU tests and the benchmark; it contains no
part of the operator or the solver.  The C source ``synth.c`` documents the
random-number streams and the SU(3) generators.  ``build()`` compiles it with
gcc; ``load()`` builds only when no shared object exists yet.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None

KIND_IDENTITY, KIND_HAAR, KIND_SMOOTH = 0, 1, 2


def build():
    cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
           "-o", _LIB + ".tmp", _SRC, "-lm"]
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
    dp = ctypes.c_void_p
    lib.synth_gauge.argtypes = [i32p, ctypes.c_int32, ctypes.c_double, ctypes.c_uint64, dp]
    lib.synth_site_haar.argtypes = [i32p, ctypes.c_uint64, dp]
    lib.synth_gauge_algebra.argtypes = [i32p, ctypes.c_uint64, dp]
    lib.synth_source.argtypes = [i32p, ctypes.c_int32, ctypes.c_uint64, dp]
    lib.synth_momenta.argtypes = [i32p, ctypes.c_uint64, dp]
    for f in (lib.synth_gauge, lib.synth_site_haar, lib.synth_gauge_algebra, lib.synth_source, lib.synth_momenta):
        f.restype = None
    _lib = lib
    return lib


def _dims(dims):
    d = np.ascontiguousarray(dims, dtype=np.int32)
    assert d.shape == (4,)
    return d, d.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def gauge(dims, kind="haar", seed=0, eps=0.3):
    """Links U[mu, t, z, y, x, a, b] as complex128, shape (4, Nt, Nz, Ny, Nx, 3, 3)."""
    k = {"identity": KIND_IDENTITY, "haar": KIND_HAAR, "smooth": KIND_SMOOTH}[kind]
    d, dp = _dims(dims)
    out = np.empty((4, d[3], d[2], d[1], d[0], 3, 3), np.complex128)
    load().synth_gauge(dp, k, float(eps), int(seed), out.ctypes.data)
    return out


def site_haar(dims, seed=0):
    """One Haar SU(3) matrix per site, shape (Nt, Nz, Ny, Nx, 3, 3)."""
    d, dp = _dims(dims)
    out = np.empty((d[3], d[2], d[1], d[0], 3, 3), np.complex128)
    load().synth_site_haar(dp, int(seed), out.ctypes.data)
    return out


def gauge_algebra(dims, seed=0):
    """The Hermitian traceless H behind gauge(kind='smooth', seed), same shape as gauge()."""
    d, dp = _dims(dims)
    out = np.empty((4, d[3], d[2], d[1], d[0], 3, 3), np.complex128)
    load().synth_gauge_algebra(dp, int(seed), out.ctypes.data)
    return out


def source(dims, parity=0, seed=0):
    """Gaussian colour vectors, shape (Nt, Nz, Ny, Nx, 3); zero off `parity` (-1: all sites)."""
    d, dp = _dims(dims)
    out = np.empty((d[3], d[2], d[1], d[0], 3), np.complex128)
    load().synth_source(dp, int(parity), int(seed), out.ctypes.data)
    return out


def momenta(dims, seed=0):
    """Anti-Hermitian traceless Q = sum_a q_a (i lambda_a / 2), q_a ~ N(0,1); same shape as gauge()."""
    d, dp = _dims(dims)
    out = np.empty((4, d[3], d[2], d[1], d[0], 3, 3), np.complex128)
    load().synth_momenta(dp, int(seed), out.ctypes.data)
    return out
