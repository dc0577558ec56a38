"""Flop and byte model of the staggered hop and of one CG iteration.

Flops: 570 per output site and right-hand side (Sec. 4.3: per direction two
complex 3x3 matrix-vector products and a vector addition), never counting
the 12-real reconstruction or the phase signs.

Bytes ("model" bytes, every neighbour read counted as in Sec. 4.3): per output
site, links_per_site links (8 here; 6 with the paper's temporal gauge) plus,
per right-hand side, 8 input and 1 output colour vectors.  A colour vector is
3 complex numbers (48 B FP64, 24 B FP32, 16 B FP16 with its float scale).
"Algorithmic" bytes count each input vector once: the minimum HBM traffic of
a hop whose neighbour reads all hit a cache.
"""

FLOPS_PER_SITE = 570
F64, F32, F16 = 0, 1, 2
_REAL = {F64: 8, F32: 4, F16: 2}
_SPINOR = {F64: 48, F32: 24, F16: 16}


def link_bytes(prec, recon=18):
    return _REAL[prec] * recon


def spinor_bytes(prec):
    return _SPINOR[prec]


def hop_model_bytes(prec, recon=18, nrhs=1, links_per_site=8):
    """Model bytes per output site of one hop applied to nrhs vectors."""
    return links_per_site * link_bytes(prec, recon) + nrhs * 9 * spinor_bytes(prec)


def hop_min_bytes(prec, recon=18, nrhs=1, links_per_site=8):
    """Bytes per output site when every input vector is fetched from memory once."""
    return links_per_site * link_bytes(prec, recon) + nrhs * 2 * spinor_bytes(prec)


def hop_flops(nrhs=1):
    return FLOPS_PER_SITE * nrhs


def arithmetic_intensity(prec, recon=18, nrhs=1, links_per_site=8):
    return hop_flops(nrhs) / hop_model_bytes(prec, recon, nrhs, links_per_site)


def cg_iteration_bytes(prec, acc_prec, recon=18, links_per_site=8):
    """Algorithmic HBM bytes per even site of one CG iteration (four kernels).

    hop t = D_oe p: links + p + t; hop q = m^2 p - D_eo t: links + t + p + q;
    update: r read and written, q read; x += alpha p and p = r + beta p: x read and
    written, r and p read, p written.
    """
    L = links_per_site * link_bytes(prec, recon)
    s, a = spinor_bytes(prec), spinor_bytes(acc_prec)
    return (L + 2 * s) + (L + 3 * s) + (2 * a + s) + (3 * a + 2 * s)
