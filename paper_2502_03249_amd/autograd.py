"""torch.autograd Functions over the library's solver and link derivative.

StaggeredSolve:  x = M^-1 b for M = m^2 - D_eo D_oe (even sites).  Backward
  solves the adjoint system M lambda = g (M is Hermitian, so this is another
  CG on the same operator), returns grad_b = lambda and the link gradient
  from the outer products of (x, lambda) (fermion_force, mode 1).
StaggeredAction: S = phi^dag M^-1 phi.  Backward returns grad_phi = 2 chi
  (chi = M^-1 phi, saved from the forward solve) and, for the links, either
  the su(3) force F = -TA(U Pi) (project=True; the HMC fermion force, the
  element of su(3) with dS/dw = Re tr(F^dag A) for U -> exp(w A) U), or the
  Euclidean gradient Pi^dag with respect to the real and imaginary parts of
  every link entry (project=False; composes with other autograd ops).

Complex gradients follow PyTorch's convention grad = dL/dRe + i dL/dIm.
Tensors: links complex128 (4, Nt, Nz, Ny, Nx, 3, 3); fields complex128
(Nt, Nz, Ny, Nx, 3) on the even sites (odd sites are ignored on input and
zero on output).  All arithmetic runs in the library's kernels.
"""
import torch

from . import F64, Field, Gauge, cg_solve, field_dot, fermion_force


def _dims_of(links):
    _, nt, nz, ny, nx, _, _ = links.shape
    return (nx, ny, nz, nt)


def _solve(ctx, gauge, mass, b, tol, max_iter, inner_prec):
    x = b.like().zero_()
    st = cg_solve(ctx, [(gauge, mass, b, x)], tol=tol, max_iter=max_iter, inner_prec=inner_prec,
                  reliable_interval=100 if inner_prec != F64 else 0)
    if st[0]["status"] != 0:
        raise RuntimeError(f"CG did not converge: {st[0]}")
    return x


class StaggeredSolve(torch.autograd.Function):
    @staticmethod
    def forward(fctx, links, b, mass, lqs_ctx, tol=1e-12, max_iter=20000, inner_prec=F64):
        dims = _dims_of(links)
        gauge = Gauge(lqs_ctx, dims, links.detach().contiguous())
        bf = Field.from_lex(lqs_ctx, b.detach().contiguous(), 0)
        xf = _solve(lqs_ctx, gauge, mass, bf, tol, max_iter, inner_prec)
        fctx.lqs = (lqs_ctx, gauge, xf, mass, tol, max_iter, inner_prec)
        return xf.to_lex(lqs_ctx)[0]

    @staticmethod
    def backward(fctx, grad_x):
        lqs_ctx, gauge, xf, mass, tol, max_iter, inner_prec = fctx.lqs
        gf = Field.from_lex(lqs_ctx, grad_x.contiguous(), 0)
        lam = _solve(lqs_ctx, gauge, mass, gf, tol, max_iter, inner_prec)
        grad_b = lam.to_lex(lqs_ctx)[0] if fctx.needs_input_grad[1] else None
        grad_links = None
        if fctx.needs_input_grad[0]:
            grad_links = fermion_force(lqs_ctx, gauge, xf, lam, coeff=1.0, mode=1)
        return grad_links, grad_b, None, None, None, None, None


class StaggeredAction(torch.autograd.Function):
    @staticmethod
    def forward(fctx, links, phi, mass, lqs_ctx, project=True, tol=1e-12, max_iter=20000, inner_prec=F64):
        dims = _dims_of(links)
        gauge = Gauge(lqs_ctx, dims, links.detach().contiguous())
        pf = Field.from_lex(lqs_ctx, phi.detach().contiguous(), 0)
        chi = _solve(lqs_ctx, gauge, mass, pf, tol, max_iter, inner_prec)
        s = field_dot(lqs_ctx, pf, chi)[0].real
        fctx.lqs = (lqs_ctx, gauge, chi, project)
        return s

    @staticmethod
    def backward(fctx, grad_s):
        lqs_ctx, gauge, chi, project = fctx.lqs
        g = float(grad_s)
        grad_phi = None
        if fctx.needs_input_grad[1]:
            grad_phi = chi.to_lex(lqs_ctx, scale=2.0 * g)[0]
        grad_links = None
        if fctx.needs_input_grad[0]:
            grad_links = fermion_force(lqs_ctx, gauge, chi, None, coeff=g, mode=0 if project else 1)
        return grad_links, grad_phi, None, None, None, None, None, None


def staggered_solve(links, b, mass, lqs_ctx, tol=1e-12, max_iter=20000, inner_prec=F64):
    return StaggeredSolve.apply(links, b, mass, lqs_ctx, tol, max_iter, inner_prec)


def staggered_action(links, phi, mass, lqs_ctx, project=True, tol=1e-12, max_iter=20000, inner_prec=F64):
    return StaggeredAction.apply(links, phi, mass, lqs_ctx, project, tol, max_iter, inner_prec)
