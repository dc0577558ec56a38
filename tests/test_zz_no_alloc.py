"""The allocation-free solve (cg_solve_noalloc) against cg_solve, through the C ABI.

Both calls launch the same kernels with the same launch shapes, so x must be
bit-identical to cg_solve's and take the same iterations; the oracle checks the
FP64 true residual of each.  Two calls in a row share the library's scratch
array: the second, smaller one must not see the first one's contents.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import field, gauge, lex_of

pytestmark = pytest.mark.gpu

lqs = pytest.importorskip("paper_2502_03249_amd")


@pytest.fixture(scope="module")
def ctx():
    c = lqs.Context(0)
    yield c
    c.close()


def _pair(ctx, dims, U, mass, b, nrhs, **kw):
    g = gauge(ctx, dims, U)
    bf = field(ctx, dims, b, 0)
    x_ref, x_na = bf.like().zero_(), bf.like()
    x_na.data.fill_(0x7F)  # garbage: the solve must not read x from zero start
    st_ref = lqs.cg_solve(ctx, [(g, mass, bf, x_ref)], **kw)
    st_na = lqs.cg_solve_noalloc(ctx, (g, mass, bf, x_na), **kw)
    torch.cuda.synchronize()
    a = lex_of(ctx, x_ref, squeeze=(nrhs == 1))
    n = lex_of(ctx, x_na, squeeze=(nrhs == 1))
    g.close()
    return a, n, st_ref, st_na


def test_noalloc_equals_cg_solve_two_calls_second_smaller(ctx):
    # first call: 8^3 x 16, two right-hand sides, FP16-storage inner with reliable updates
    dims, mass = (8, 8, 8, 16), 0.05
    U = synth.gauge(dims, "smooth", seed=1004, eps=0.3)
    b = np.stack([synth.source(dims, 0, seed=2100 + k) for k in range(2)])
    a, n, st_ref, st_na = _pair(ctx, dims, U, mass, b, 2, tol=1e-10, inner_prec=lqs.F16, inner_recon=12)
    assert np.array_equal(a, n)
    for k in range(2):
        assert st_na[k]["status"] == 0 and st_na[k]["iters"] == st_ref[k]["iters"]
        assert st_na[k]["reliable_updates"] == st_ref[k]["reliable_updates"]
        assert oracle.true_residual(dims, U, mass, b[k], n[k]) <= 1e-10

    # second call, smaller: 4^4 FP64 (its workspace starts where the first one's did)
    dims, mass = (4, 4, 4, 4), 0.1
    U = synth.gauge(dims, "haar", seed=1000)
    b = synth.source(dims, 0, seed=2000)
    a, n, st_ref, st_na = _pair(ctx, dims, U, mass, b, 1, tol=1e-10)
    assert np.array_equal(a, n)
    assert st_na[0]["status"] == 0 and st_na[0]["iters"] == st_ref[0]["iters"]
    assert oracle.true_residual(dims, U, mass, b, n) <= 1e-10


def test_noalloc_rejects_a_problem_beyond_the_scratch_array(ctx):
    # 16^4 with 16 FP64 right-hand sides needs about 100 MB of workspace (> 64 MiB)
    dims = (16, 16, 16, 16)
    U = synth.gauge(dims, "haar", seed=1031)
    g = gauge(ctx, dims, U, lqs.fmt(lqs.F64, 18))
    b = lqs.Field(dims, lqs.F64, 0, 16).zero_()
    x = b.like().zero_()
    with pytest.raises(lqs.LqsError) as e:
        lqs.cg_solve_noalloc(ctx, (g, 0.1, b, x))
    assert e.value.status == lqs.EINVAL and "scratch" in str(e.value)
    g.close()
