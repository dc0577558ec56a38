"""Helpers for GPU tests: move seeded inputs to the device, wrap them in the
library's objects, and bring results back in the oracle's layout."""
import numpy as np
import torch

import paper_2502_03249_amd as lqs


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def gauge(ctx, dims, U, formats=lqs.FMT_ALL):
    Ud = dev(U)
    g = lqs.Gauge(ctx, dims, Ud, formats)
    g._links = Ud
    return g


def field(ctx, dims, lex, parity, prec=lqs.F64):
    """lex: numpy complex128 (Nt,Nz,Ny,Nx,3) or (nrhs,Nt,Nz,Ny,Nx,3)."""
    return lqs.Field.from_lex(ctx, dev(lex), parity, prec)


def lex_of(ctx, f, squeeze=True):
    out = host(f.to_lex(ctx))
    return out[0] if squeeze and out.shape[0] == 1 else out


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
