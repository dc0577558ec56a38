"""Error paths of the C ABI with a live context: invalid arguments are rejected
before any launch, missing formats are reported, non-finite input is caught."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from gpu_util import dev, field, gauge

pytestmark = pytest.mark.gpu

lqs = pytest.importorskip("paper_2502_03249_amd")


@pytest.fixture(scope="module")
def setup():
    ctx = lqs.Context(0)
    dims = (4, 4, 4, 8)
    U = synth.gauge(dims, "haar", seed=1)
    g_all = gauge(ctx, dims, U)
    g64 = gauge(ctx, dims, U, lqs.fmt(lqs.F64, 18))
    src = synth.source(dims, -1, seed=2)
    yield ctx, dims, U, g_all, g64, src
    ctx.close()


def _status(fn):
    with pytest.raises(lqs.LqsError) as e:
        fn()
    return e.value.status


def test_hop_argument_checks(setup):
    ctx, dims, U, g, g64, src = setup
    x = field(ctx, dims, src, 1)
    same = x.like(parity=1)
    assert _status(lambda: lqs.dslash_apply(ctx, g, x, same)) == lqs.EINVAL          # parities
    assert _status(lambda: lqs.dslash_apply(ctx, g, x, x.like(parity=0, prec=lqs.F32))) == lqs.EINVAL
    assert _status(lambda: lqs.dslash_apply(ctx, g, x, recon=13)) == lqs.EINVAL
    alias = lqs.Field(dims, lqs.F64, 0, 1, data=x.data)
    assert _status(lambda: lqs.dslash_apply(ctx, g, x, alias)) == lqs.EINVAL           # overlap
    xh = field(ctx, dims, src, 1, lqs.F16)
    assert _status(lambda: lqs.dslash_apply(ctx, g64, xh)) == lqs.EUNSUPPORTED         # format absent
    x2 = field(ctx, dims, np.stack([src, src]), 1)
    assert _status(lambda: lqs.dslash_apply(ctx, g, x2, x.like(parity=0))) == lqs.EINVAL  # nrhs


def test_misaligned_pointer_rejected(setup):
    ctx, dims, U, g, g64, src = setup
    x = field(ctx, dims, src, 1)
    raw = torch.empty(x.data.numel() + 64, dtype=torch.uint8, device="cuda")
    bad = lqs.Field(dims, lqs.F64, 0, 1, data=raw[8:8 + x.data.numel()])
    assert _status(lambda: lqs.dslash_apply(ctx, g, x, bad)) == lqs.EINVAL


def test_cg_parameter_checks(setup):
    ctx, dims, U, g, g64, src = setup
    b = field(ctx, dims, src, 0)
    x = b.like()
    assert _status(lambda: lqs.cg_solve(ctx, [(g, 0.1, b, x)], tol=0.0)) == lqs.EINVAL
    assert _status(lambda: lqs.cg_solve(ctx, [(g, 0.1, b, x)], max_iter=0)) == lqs.EINVAL
    assert _status(lambda: lqs.cg_solve(ctx, [(g, 0.1, b, x)], inner_recon=8)) == lqs.EINVAL
    assert _status(lambda: lqs.cg_solve(ctx, [(g, -1.0, b, x)])) == lqs.EINVAL
    assert _status(lambda: lqs.cg_solve(ctx, [(g64, 0.1, b, x)], inner_prec=lqs.F16)) == lqs.EUNSUPPORTED
    assert _status(lambda: lqs.fermion_force(ctx, g, b, None, 1.0, mode=3)) == lqs.EINVAL
    # an empty batch: no problem to solve is an argument error, not a silent success
    L = lqs.lib()
    prm = lqs.LqsCgParams(1e-10, 100, lqs.F64, 18, 0, 0.0, 0, 0)
    stats = (lqs.LqsCgStats * 1)()
    assert L.cg_solve(ctx.handle, 0, None, ctypes.byref(prm), stats, None) == lqs.EINVAL


def test_nonfinite_source_reported(setup):
    ctx, dims, U, g, g64, src = setup
    s = synth.source(dims, 0, seed=3)
    s[0, 0, 0, 0, 1] = np.nan
    b = field(ctx, dims, s, 0)
    x = b.like()
    st = lqs.cg_solve(ctx, [(g, 0.1, b, x.zero_())], tol=1e-10)
    assert st[0]["status"] == lqs.ENONFINITE


def test_gauge_rejects_odd_extent(setup):
    ctx, dims, U, g, g64, src = setup
    bad = (4, 4, 5, 8)
    links = torch.zeros((4, 8, 5, 4, 4, 3, 3), dtype=torch.complex128, device="cuda")
    h = ctypes.c_void_p()
    st = lqs.lib().lqs_gauge_create(ctx.handle, (ctypes.c_int32 * 4)(*bad), ctypes.c_void_p(links.data_ptr()),
                                    lqs.FMT_ALL, None, ctypes.byref(h))
    assert st == lqs.EINVAL
