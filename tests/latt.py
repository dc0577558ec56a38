"""Lattice helpers for the tests (numpy, test side only).

Arrays follow the canonical layout: fields (Nt, Nz, Ny, Nx, 3), links
(4, Nt, Nz, Ny, Nx, 3, 3); direction mu = 0..3 is x..t, so the array axis of
direction mu is 3 - mu.  dims = (Nx, Ny, Nz, Nt).
"""
import numpy as np


def axis(mu):
    return 3 - mu


def coords(dims):
    nx, ny, nz, nt = dims
    t, z, y, x = np.meshgrid(np.arange(nt), np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x, y, z, t


def parity_mask(dims, p):
    x, y, z, t = coords(dims)
    return ((x + y + z + t) % 2) == p


def on_parity(f, dims, p):
    """Zero f off the sites of parity p."""
    return f * parity_mask(dims, p)[..., None]


def shift(f, mu, step):
    """g(x) = f(x + step*mu-hat), periodic wrap (no boundary sign)."""
    return np.roll(f, -step, axis=axis(mu))


def gauge_transform(U, G):
    """U^G_{x,mu} = G_x U_{x,mu} G^dag_{x+mu}."""
    out = np.empty_like(U)
    for mu in range(4):
        Gf = shift(G, mu, 1)
        out[mu] = G @ U[mu] @ np.conj(np.swapaxes(Gf, -1, -2))
    return out


def apply_site(G, f):
    """(G f)(x) = G_x f(x)."""
    return np.einsum("...ab,...b->...a", G, f)


def plane_wave(dims, n, colour, p_mask=None):
    """exp(i p.x) * colour, p_i = 2 pi n_i / N_i (i = x,y,z), p_t = (2 n_t + 1) pi / N_t."""
    nx, ny, nz, nt = dims
    x, y, z, t = coords(dims)
    p = (2 * np.pi * n[0] / nx, 2 * np.pi * n[1] / ny, 2 * np.pi * n[2] / nz, (2 * n[3] + 1) * np.pi / nt)
    ph = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    return ph[..., None] * np.asarray(colour)[None, None, None, None, :], p


def free_momenta(dims):
    nx, ny, nz, nt = dims
    out = []
    for a in range(nx):
        for b in range(ny):
            for c in range(nz):
                for d in range(nt):
                    out.append((2 * np.pi * a / nx, 2 * np.pi * b / ny, 2 * np.pi * c / nz, (2 * d + 1) * np.pi / nt))
    return np.array(out)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def su3_generators():
    """A_a = i lambda_a / 2 (Gell-Mann), a basis of su(3)."""
    l = np.zeros((8, 3, 3), np.complex128)
    l[0][0, 1] = l[0][1, 0] = 1
    l[1][0, 1], l[1][1, 0] = -1j, 1j
    l[2][0, 0], l[2][1, 1] = 1, -1
    l[3][0, 2] = l[3][2, 0] = 1
    l[4][0, 2], l[4][2, 0] = -1j, 1j
    l[5][1, 2] = l[5][2, 1] = 1
    l[6][1, 2], l[6][2, 1] = -1j, 1j
    l[7][0, 0] = l[7][1, 1] = 1 / np.sqrt(3)
    l[7][2, 2] = -2 / np.sqrt(3)
    return 0.5j * l


def expm_su3(A):
    """exp of a small 3x3 matrix (eigendecomposition; A anti-Hermitian)."""
    w, v = np.linalg.eigh(-1j * A)
    return v @ np.diag(np.exp(1j * w)) @ np.conj(v.T)
