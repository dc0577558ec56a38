"""MI355X staggered-fermion solver: Python binding of liblqs.so.

The binding only marshals arguments to the C ABI declared in include/lqs.h
(ctypes; torch supplies device memory and the HIP stream).  Every step of the
operator and the solver runs in the library's HIP kernels; there is no Python
or CPU fallback, and importing a function that needs the library raises if
liblqs.so has not been built (``paper_2502_03249_amd.build.build()``).

Names follow the C ABI: dslash_apply, dslash_dagger, cg_solve, fermion_force.
dims = (Nx, Ny, Nz, Nt); canonical complex128 layouts are links
(4, Nt, Nz, Ny, Nx, 3, 3) and colour-vector fields (nrhs, Nt, Nz, Ny, Nx, 3).
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblqs.so")

F64, F32, F16 = 0, 1, 2
PREC = {"f64": F64, "f32": F32, "f16": F16, F64: F64, F32: F32, F16: F16}

OK, ENOTCONV, EINVAL, EHIP, ENOMEM, EBREAKDOWN, ENONFINITE, EUNSUPPORTED = 0, 1, -1, -2, -3, -4, -5, -6


def fmt(prec, recon):
    """Format bit of LQS_FMT(prec, recon)."""
    return 1 << (2 * PREC[prec] + (1 if recon == 12 else 0))


FMT_ALL = 0x3F
TEMPORAL_GAUGE = 0x100


class LqsField(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("prec", ctypes.c_int32), ("parity", ctypes.c_int32),
                ("nrhs", ctypes.c_int32)]


class LqsProblem(ctypes.Structure):
    _fields_ = [("gauge", ctypes.c_void_p), ("mass", ctypes.c_double), ("nrhs", ctypes.c_int32),
                ("b", ctypes.c_void_p), ("x", ctypes.c_void_p)]


class LqsCgParams(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("inner_prec", ctypes.c_int32),
                ("inner_recon", ctypes.c_int32), ("reliable_interval", ctypes.c_int32),
                ("reliable_delta", ctypes.c_double), ("use_x0", ctypes.c_int32), ("persistent", ctypes.c_int32)]


class LqsCgStats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("reliable_updates", ctypes.c_int32),
                ("restarts", ctypes.c_int32), ("true_rel_residual", ctypes.c_double), ("seconds", ctypes.c_double),
                ("device_seconds", ctypes.c_double), ("gflops", ctypes.c_double), ("gbytes_per_s", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class LqsHmcParams(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("mass", ctypes.c_double), ("tau", ctypes.c_double),
                ("nsteps", ctypes.c_int32), ("integrator", ctypes.c_int32), ("lam", ctypes.c_double),
                ("fermions", ctypes.c_int32), ("cg", LqsCgParams), ("force_tol", ctypes.c_double)]


class LqsHmcStats(ctypes.Structure):
    _fields_ = [("k0", ctypes.c_double), ("sg0", ctypes.c_double), ("sf0", ctypes.c_double),
                ("k1", ctypes.c_double), ("sg1", ctypes.c_double), ("sf1", ctypes.c_double),
                ("dH", ctypes.c_double), ("accepted", ctypes.c_int32), ("cg_solves", ctypes.c_int32),
                ("cg_iters", ctypes.c_int32), ("status", ctypes.c_int32), ("plaquette", ctypes.c_double),
                ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


LEAPFROG, OMELYAN = 0, 1


class LqsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"lqs status {status}: {msg}")
        self.status = status


_lib = None
EXPORTS = ["lqs_ctx_create", "lqs_ctx_destroy", "lqs_set_tuning", "lqs_gauge_create", "lqs_gauge_destroy",
           "lqs_field_bytes", "lqs_field_pack", "lqs_field_unpack", "dslash_apply", "dslash_dagger", "cg_solve",
           "fermion_force", "lqs_strerror", "lqs_last_error", "lqs_profile_hops", "lqs_profile_hops_result",
           "lqs_field_dot", "cg_solve_multishift", "lqs_gauge_fix_temporal", "gauge_action", "gauge_force",
           "link_update", "kinetic_energy", "hmc_trajectory", "lqs_set_graphs", "lqs_field_unpack_scaled",
           "cg_solve_noalloc"]


def lib():
    """The loaded liblqs.so (torch's HIP runtime is loaded first and shared)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2502_03249_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    i32p = ctypes.POINTER(ctypes.c_int32)
    L.lqs_ctx_create.argtypes = [i32, ctypes.c_char_p, ctypes.POINTER(vp)]
    L.lqs_ctx_destroy.argtypes = [vp]
    L.lqs_ctx_destroy.restype = None
    L.lqs_set_tuning.argtypes = [vp, i32]
    L.lqs_set_graphs.argtypes = [vp, i32]
    L.lqs_gauge_create.argtypes = [vp, i32p, vp, ctypes.c_uint32, vp, ctypes.POINTER(vp)]
    L.lqs_gauge_destroy.argtypes = [vp]
    L.lqs_gauge_destroy.restype = None
    L.lqs_field_bytes.argtypes = [i32p, i32, i32, ctypes.POINTER(ctypes.c_size_t)]
    L.lqs_gauge_fix_temporal.argtypes = [vp, i32p, vp, vp, vp, vp]
    L.lqs_field_pack.argtypes = [vp, i32p, vp, ctypes.POINTER(LqsField), vp]
    L.lqs_field_unpack.argtypes = [vp, i32p, ctypes.POINTER(LqsField), vp, vp]
    L.lqs_field_unpack_scaled.argtypes = [vp, i32p, ctypes.POINTER(LqsField), d, vp, vp]
    L.dslash_apply.argtypes = [vp, vp, i32, ctypes.POINTER(LqsField), ctypes.POINTER(LqsField), vp]
    L.dslash_dagger.argtypes = [vp, vp, i32, ctypes.POINTER(LqsField), ctypes.POINTER(LqsField), vp]
    L.cg_solve.argtypes = [vp, i32, ctypes.POINTER(LqsProblem), ctypes.POINTER(LqsCgParams),
                           ctypes.POINTER(LqsCgStats), vp]
    L.cg_solve_noalloc.argtypes = [vp, ctypes.POINTER(LqsProblem), ctypes.POINTER(LqsCgParams),
                                   ctypes.POINTER(LqsCgStats), vp]
    L.fermion_force.argtypes = [vp, vp, vp, vp, d, i32, vp, vp]
    L.cg_solve_multishift.argtypes = [vp, vp, i32, ctypes.POINTER(d), vp, ctypes.POINTER(vp),
                                      ctypes.POINTER(LqsCgParams), ctypes.POINTER(LqsCgStats), vp]
    L.lqs_strerror.argtypes = [i32]
    L.lqs_strerror.restype = ctypes.c_char_p
    L.lqs_last_error.argtypes = []
    L.lqs_last_error.restype = ctypes.c_char_p
    L.lqs_field_dot.argtypes = [vp, i32p, ctypes.POINTER(LqsField), ctypes.POINTER(LqsField), vp, vp]
    L.lqs_profile_hops.argtypes = [vp, i32]
    L.gauge_action.argtypes = [vp, i32p, vp, d, ctypes.POINTER(d), vp]
    L.gauge_force.argtypes = [vp, i32p, vp, d, d, i32, vp, vp]
    L.link_update.argtypes = [vp, i32p, vp, vp, d, vp]
    L.kinetic_energy.argtypes = [vp, i32p, vp, ctypes.POINTER(d), vp]
    L.hmc_trajectory.argtypes = [vp, i32p, vp, vp, vp, d, ctypes.POINTER(LqsHmcParams), ctypes.POINTER(LqsHmcStats),
                                 vp, vp, vp]
    L.lqs_profile_hops_result.argtypes = [vp, i32, i32, d, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(d),
                                          ctypes.POINTER(ctypes.c_int64)]
    for name in EXPORTS:
        f = getattr(L, name)
        if name not in ("lqs_ctx_destroy", "lqs_gauge_destroy", "lqs_strerror", "lqs_last_error"):
            f.restype = i32
    _lib = L
    return L


def _check(status, allow_warning=False):
    if status == OK or (allow_warning and status > 0):
        return status
    L = lib()
    raise LqsError(status, f"{L.lqs_strerror(status).decode()}: {L.lqs_last_error().decode()}")


def _dims(dims):
    arr = (ctypes.c_int32 * 4)(*[int(v) for v in dims])
    return arr


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Context:
    """Library context on one device (workspace, tuning cache)."""

    def __init__(self, device=0, tune_cache=None, tuning=False):
        self.device = int(device)
        h = ctypes.c_void_p()
        _check(lib().lqs_ctx_create(self.device, tune_cache.encode() if tune_cache else None, ctypes.byref(h)))
        self.handle = h
        if tuning:
            _check(lib().lqs_set_tuning(self.handle, 1))

    def set_tuning(self, enable):
        _check(lib().lqs_set_tuning(self.handle, 1 if enable else 0))

    def set_graphs(self, enable):
        _check(lib().lqs_set_graphs(self.handle, 1 if enable else 0))

    def close(self):
        if getattr(self, "handle", None):
            torch.cuda.synchronize(self.device)
            lib().lqs_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def torch_device(self):
        return torch.device("cuda", self.device)


def field_bytes(dims, prec, nrhs=1):
    n = ctypes.c_size_t()
    _check(lib().lqs_field_bytes(_dims(dims), PREC[prec], int(nrhs), ctypes.byref(n)))
    return int(n.value)


class Gauge:
    """Packed copies of one gauge field (links: canonical complex128 on the device)."""

    def __init__(self, ctx, dims, links, formats=FMT_ALL, stream=None):
        assert links.is_cuda and links.dtype == torch.complex128 and links.is_contiguous()
        nx, ny, nz, nt = dims
        assert tuple(links.shape) == (4, nt, nz, ny, nx, 3, 3)
        self.ctx = ctx
        self.dims = tuple(int(v) for v in dims)
        h = ctypes.c_void_p()
        _check(lib().lqs_gauge_create(ctx.handle, _dims(dims), ctypes.c_void_p(links.data_ptr()), int(formats),
                                      _stream(stream), ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().lqs_gauge_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gauge_fix_temporal(ctx, dims, links, stream=None):
    """Temporal gauge (U_t = 1 off the last slice): returns (fixed links, G), canonical complex128 tensors."""
    assert links.is_cuda and links.dtype == torch.complex128 and links.is_contiguous()
    out = torch.empty_like(links)
    G = torch.empty(links.shape[1:], dtype=torch.complex128, device=links.device)
    _check(lib().lqs_gauge_fix_temporal(ctx.handle, _dims(dims), ctypes.c_void_p(links.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(G.data_ptr()),
                                        _stream(stream)))
    return out, G


class Field:
    """A native single-parity field of nrhs right-hand sides (device memory owned by torch)."""

    def __init__(self, dims, prec, parity, nrhs=1, device=0, data=None):
        self.dims = tuple(int(v) for v in dims)
        self.prec = PREC[prec]
        self.parity = int(parity)
        self.nrhs = int(nrhs)
        nbytes = field_bytes(self.dims, self.prec, self.nrhs)
        if data is None:
            data = torch.empty(nbytes, dtype=torch.uint8, device=torch.device("cuda", device))
        assert data.is_cuda and data.numel() * data.element_size() >= nbytes and data.is_contiguous()
        self.data = data

    def c(self):
        return LqsField(ctypes.c_void_p(self.data.data_ptr()), self.prec, self.parity, self.nrhs)

    def like(self, parity=None, prec=None):
        return Field(self.dims, self.prec if prec is None else prec, self.parity if parity is None else parity,
                     self.nrhs, self.data.device.index)

    def zero_(self):
        self.data.zero_()
        return self

    @property
    def f64(self):
        """FP64 fields as float64 view, shape (nrhs, 3, Vh, 2)."""
        assert self.prec == F64
        nx, ny, nz, nt = self.dims
        return self.data.view(torch.float64).view(self.nrhs, 3, nx * ny * nz * nt // 2, 2)

    @staticmethod
    def from_lex(ctx, lex, parity, prec=F64, stream=None):
        """Pack canonical complex128 (nrhs, Nt, Nz, Ny, Nx, 3) or (Nt, Nz, Ny, Nx, 3); reads only `parity` sites."""
        assert lex.is_cuda and lex.dtype == torch.complex128
        if lex.dim() == 5:
            lex = lex.unsqueeze(0)
        lex = lex.contiguous()
        nrhs, nt, nz, ny, nx, _ = lex.shape
        f = Field((nx, ny, nz, nt), prec, parity, nrhs, lex.device.index)
        c = f.c()
        _check(lib().lqs_field_pack(ctx.handle, _dims(f.dims), ctypes.c_void_p(lex.data_ptr()), ctypes.byref(c),
                                    _stream(stream)))
        f._keep = lex
        return f

    def to_lex(self, ctx, out=None, stream=None, scale=None):
        """Unpack into canonical complex128 (nrhs, Nt, Nz, Ny, Nx, 3), zero off this field's parity;
        with scale, every value is multiplied by that real number inside the library."""
        nx, ny, nz, nt = self.dims
        if out is None:
            out = torch.zeros((self.nrhs, nt, nz, ny, nx, 3), dtype=torch.complex128, device=self.data.device)
        c = self.c()
        if scale is None:
            _check(lib().lqs_field_unpack(ctx.handle, _dims(self.dims), ctypes.byref(c),
                                          ctypes.c_void_p(out.data_ptr()), _stream(stream)))
        else:
            _check(lib().lqs_field_unpack_scaled(ctx.handle, _dims(self.dims), ctypes.byref(c), float(scale),
                                                 ctypes.c_void_p(out.data_ptr()), _stream(stream)))
        return out


def _hop(fn, ctx, gauge, x, out, recon, stream):
    if out is None:
        out = x.like(parity=1 - x.parity)
    ci, co = x.c(), out.c()
    _check(fn(ctx.handle, gauge.handle, int(recon), ctypes.byref(ci), ctypes.byref(co), _stream(stream)))
    return out


def dslash_apply(ctx, gauge, x, out=None, recon=18, stream=None):
    """out = D_{p,1-p} x (eq. (1) at the sites of the other parity)."""
    return _hop(lib().dslash_apply, ctx, gauge, x, out, recon, stream)


def dslash_dagger(ctx, gauge, x, out=None, recon=18, stream=None):
    """out = (D^dag)_{p,1-p} x."""
    return _hop(lib().dslash_dagger, ctx, gauge, x, out, recon, stream)


def cg_solve(ctx, problems, tol=1e-10, max_iter=10000, inner_prec=F64, inner_recon=18, reliable_interval=0,
             reliable_delta=0.0, use_x0=False, persistent=False, stream=None):
    """Solve M x = b for each (gauge, mass, b, x) with b, x FP64 even Fields; returns per-rhs stats dicts."""
    n = len(problems)
    arr = (LqsProblem * n)()
    total = 0
    for i, (g, m, b, x) in enumerate(problems):
        assert b.prec == F64 and x.prec == F64 and b.parity == 0 and x.parity == 0 and b.nrhs == x.nrhs
        arr[i] = LqsProblem(g.handle, float(m), b.nrhs, ctypes.c_void_p(b.data.data_ptr()),
                            ctypes.c_void_p(x.data.data_ptr()))
        total += b.nrhs
    prm = LqsCgParams(float(tol), int(max_iter), PREC[inner_prec], int(inner_recon), int(reliable_interval),
                      float(reliable_delta), 1 if use_x0 else 0, 1 if persistent else 0)
    stats = (LqsCgStats * total)()
    st = lib().cg_solve(ctx.handle, n, arr, ctypes.byref(prm), stats, _stream(stream))
    if st < 0 and st not in (EBREAKDOWN, ENONFINITE):
        _check(st)
    return [s.as_dict() for s in stats]


def cg_solve_noalloc(ctx, problem, tol=1e-10, max_iter=10000, inner_prec=F64, inner_recon=18, reliable_interval=0,
                     reliable_delta=0.0, use_x0=False, stream=None):
    """cg_solve of one (gauge, mass, b, x) problem with the library's fixed scratch array as workspace (no device
    allocation inside the call); returns per-rhs stats dicts."""
    g, m, b, x = problem
    assert b.prec == F64 and x.prec == F64 and b.parity == 0 and x.parity == 0 and b.nrhs == x.nrhs
    pb = LqsProblem(g.handle, float(m), b.nrhs, ctypes.c_void_p(b.data.data_ptr()), ctypes.c_void_p(x.data.data_ptr()))
    prm = LqsCgParams(float(tol), int(max_iter), PREC[inner_prec], int(inner_recon), int(reliable_interval),
                      float(reliable_delta), 1 if use_x0 else 0, 0)
    stats = (LqsCgStats * b.nrhs)()
    st = lib().cg_solve_noalloc(ctx.handle, ctypes.byref(pb), ctypes.byref(prm), stats, _stream(stream))
    if st < 0 and st not in (EBREAKDOWN, ENONFINITE):
        _check(st)
    return [s.as_dict() for s in stats]


def cg_solve_multishift(ctx, gauge, masses, b, xs, tol=1e-10, max_iter=10000, inner_prec=F64, inner_recon=18,
                        reliable_interval=0, reliable_delta=0.0, stream=None):
    """x_i = (m_i^2 - D_eo D_oe)^-1 b for every mass on one Krylov space (recurrence in inner_prec, solutions
    in FP64, per-mass FP64 check and refinement); returns per-mass stats."""
    n = len(masses)
    assert len(xs) == n and b.prec == F64 and b.parity == 0 and b.nrhs == 1
    for x in xs:
        assert x.prec == F64 and x.parity == 0 and x.nrhs == 1
    m = (ctypes.c_double * n)(*[float(v) for v in masses])
    ptrs = (ctypes.c_void_p * n)(*[x.data.data_ptr() for x in xs])
    prm = LqsCgParams(float(tol), int(max_iter), PREC[inner_prec], int(inner_recon), int(reliable_interval),
                      float(reliable_delta), 0, 0)
    stats = (LqsCgStats * n)()
    st = lib().cg_solve_multishift(ctx.handle, gauge.handle, n, m, ctypes.c_void_p(b.data.data_ptr()), ptrs,
                                   ctypes.byref(prm), stats, _stream(stream))
    if st < 0 and st not in (EBREAKDOWN, ENONFINITE):
        _check(st)
    return [s.as_dict() for s in stats]


def fermion_force(ctx, gauge, X, Y=None, coeff=1.0, mode=0, out=None, stream=None):
    """Link derivative (mode 0: su(3) force, mode 1: Euclidean gradient), canonical complex128 links."""
    nx, ny, nz, nt = gauge.dims
    if out is None:
        out = torch.empty((4, nt, nz, ny, nx, 3, 3), dtype=torch.complex128, device=X.data.device)
    assert X.prec == F64 and X.parity == 0 and X.nrhs == 1
    yp = None
    if Y is not None:
        assert Y.prec == F64 and Y.parity == 0 and Y.nrhs == 1
        yp = ctypes.c_void_p(Y.data.data_ptr())
    _check(lib().fermion_force(ctx.handle, gauge.handle, ctypes.c_void_p(X.data.data_ptr()), yp, float(coeff),
                               int(mode), ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def field_dot(ctx, a, b, out=None, stream=None):
    """sum_sites a^dag b per right-hand side (FP64 fields) as a complex128 device tensor of nrhs entries."""
    assert a.prec == F64 and b.prec == F64
    if out is None:
        out = torch.empty(a.nrhs, dtype=torch.complex128, device=a.data.device)
    ca, cb = a.c(), b.c()
    _check(lib().lqs_field_dot(ctx.handle, _dims(a.dims), ctypes.byref(ca), ctypes.byref(cb),
                               ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def _links_tensor(dims, t, what):
    nx, ny, nz, nt = dims
    assert t.dtype == torch.complex128 and t.is_contiguous() and tuple(t.shape) == (4, nt, nz, ny, nx, 3, 3), what
    return ctypes.c_void_p(t.data_ptr())


def gauge_action(ctx, dims, links, beta, stream=None):
    """S_g = beta sum_x sum_{mu<nu} (1 - Re tr P / 3) of complex128 links (4, Nt, Nz, Ny, Nx, 3, 3)."""
    S = ctypes.c_double()
    _check(lib().gauge_action(ctx.handle, _dims(dims), _links_tensor(dims, links, "links"), float(beta),
                              ctypes.byref(S), _stream(stream)))
    return float(S.value)


def gauge_force(ctx, dims, links, beta, coeff=1.0, out=None, accumulate=False, stream=None):
    """coeff * (beta/3) TA(U V) per link (out = or out +=); returns out."""
    if out is None:
        out = torch.empty_like(links)
    _check(lib().gauge_force(ctx.handle, _dims(dims), _links_tensor(dims, links, "links"), float(beta), float(coeff),
                             1 if accumulate else 0, _links_tensor(dims, out, "out"), _stream(stream)))
    return out


def link_update(ctx, dims, links, mom, eps, stream=None):
    """links = exp(eps Q) links in place; returns links."""
    _check(lib().link_update(ctx.handle, _dims(dims), _links_tensor(dims, links, "links"),
                             _links_tensor(dims, mom, "mom"), float(eps), _stream(stream)))
    return links


def kinetic_energy(ctx, dims, mom, stream=None):
    """K = -sum_links tr Q^2."""
    K = ctypes.c_double()
    _check(lib().kinetic_energy(ctx.handle, _dims(dims), _links_tensor(dims, mom, "mom"), ctypes.byref(K),
                                _stream(stream)))
    return float(K.value)


def hmc_trajectory(ctx, dims, links, mom, pf=None, u=0.5, beta=5.5, mass=0.1, tau=1.0, nsteps=10,
                   integrator=LEAPFROG, lam=0.0, fermions=1, tol=1e-10, max_iter=10000, inner_prec=F64,
                   inner_recon=18, reliable_interval=0, reliable_delta=0.0, use_x0=False, force_tol=0.0,
                   proposal=None, phi_out=None, stream=None, check=True):
    """One HMC trajectory on complex128 links/momenta (updated in place); pf: eta (fermions=1) or phi
    (fermions=2) as a complex128 lex tensor (Nt, Nz, Ny, Nx, 3).  Returns the stats dict."""
    nx, ny, nz, nt = dims
    p = LqsHmcParams(float(beta), float(mass), float(tau), int(nsteps), int(integrator), float(lam), int(fermions),
                     LqsCgParams(float(tol), int(max_iter), PREC[inner_prec], int(inner_recon),
                                 int(reliable_interval), float(reliable_delta), 1 if use_x0 else 0, 0),
                     float(force_tol))
    st = LqsHmcStats()
    pfp = None
    if fermions:
        assert pf is not None and pf.dtype == torch.complex128 and pf.is_contiguous()
        assert tuple(pf.shape) == (nt, nz, ny, nx, 3)
        pfp = ctypes.c_void_p(pf.data_ptr())
    prop = _links_tensor(dims, proposal, "proposal") if proposal is not None else None
    po = None
    if phi_out is not None:
        assert phi_out.dtype == torch.complex128 and tuple(phi_out.shape) == (nt, nz, ny, nx, 3)
        po = ctypes.c_void_p(phi_out.data_ptr())
    r = lib().hmc_trajectory(ctx.handle, _dims(dims), _links_tensor(dims, links, "links"),
                             _links_tensor(dims, mom, "mom"), pfp, float(u), ctypes.byref(p), ctypes.byref(st),
                             prop, po, _stream(stream))
    if check and r < 0:
        _check(r)
    d = st.as_dict()
    d["return_status"] = int(r)
    return d


def profile_hops(ctx, enable):
    _check(lib().lqs_profile_hops(ctx.handle, 1 if enable else 0))


def profile_hops_result(ctx, prec, recon, min_ms=0.0):
    n, ms, sites = ctypes.c_int64(), ctypes.c_double(), ctypes.c_int64()
    _check(lib().lqs_profile_hops_result(ctx.handle, PREC[prec], int(recon), float(min_ms), ctypes.byref(n),
                                         ctypes.byref(ms),
                                         ctypes.byref(sites)))
    return int(n.value), float(ms.value), int(sites.value)
