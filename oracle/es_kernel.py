"""Exponential-of-semicircle (ES) convolution kernel and its gridding
correction, in FP64.

The paper delegates de/gridding to an external gridder (Section 2 and
Section 5.3) and names no kernel.  The ES kernel is the one of the CPU
gridding work the paper cites in Section 2 (Barnett et al. 2019):

    phi(z) = exp(beta * (sqrt(1 - z^2) - 1))   for |z| <= 1, else 0,

stretched over W grid cells: the weight of cell c for a visibility at grid
coordinate x is phi((c - x) / (W/2)).  Reading: beta = 2.30 W,
the value that reference publishes for upsampling factor 2.

The W cells used for coordinate x are floor(x) - W/2 + 1 ... floor(x) + W/2
(so at an exact integer x the left cell with phi(-1) is the excluded one).

The gridding correction is the continuous Fourier transform of the stretched
kernel evaluated at the image pixel offsets p = ix - N/2 (cycles per grid
cell p / Ng):

    psi_hat(p) = (W/2) * integral_{-1}^{1} phi(z) cos(pi * W * z * p / Ng) dz

computed here with Gauss-Legendre quadrature (default 256 nodes).
"""

import numpy as np


def es_beta(support):
    """beta = 2.30 * W (reading for upsampling factor sigma = 2)."""
    return 2.30 * float(support)


def es_phi(z, beta):
    """phi(z) = exp(beta (sqrt(1 - z^2) - 1)) on |z| <= 1, zero outside."""
    z = np.asarray(z, dtype=np.float64)
    out = np.zeros(z.shape, dtype=np.float64)
    inside = np.abs(z) <= 1.0
    out[inside] = np.exp(beta * (np.sqrt(1.0 - z[inside] ** 2) - 1.0))
    return out


def taps(x, support, beta):
    """First tap cell and the W tap weights for grid coordinates ``x``.

    Returns ``first`` (int64, shape x.shape) and ``w`` (float64,
    shape x.shape + (W,)), with w[..., i] the weight of cell first + i.
    """
    x = np.asarray(x, dtype=np.float64)
    first = np.floor(x).astype(np.int64) - support // 2 + 1
    dist = (first[..., None] + np.arange(support)) - x[..., None]  # c - x
    return first, es_phi(dist / (support / 2.0), beta)


def correction(n_img, n_grid, support, beta, nodes=256):
    """psi_hat(p) for the N pixel offsets p = ix - N/2 of one image axis."""
    z, wq = np.polynomial.legendre.leggauss(nodes)
    p = np.arange(n_img, dtype=np.float64) - n_img // 2
    phase = np.pi * support * np.outer(p, z) / n_grid
    return (support / 2.0) * (np.cos(phase) @ (wq * es_phi(z, beta)))
