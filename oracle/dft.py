"""Direct Fourier sums: the plain definition of the measurement operator.

Eq. 1 (Section 2) with the direction-independent and direction-dependent
terms set to one and the w term dropped reduces, as Section 2 states, to a
two-dimensional Fourier transform.  Reading: the 1/n factor is
dropped too, and the sky is the pixelised model image, so

    (A x)_k  = sum_p x_p exp(-2 pi i (u_k l_p + v_k m_p))      (forward)
    (A^H y)_p = sum_k y_k exp(+2 pi i (u_k l_p + v_k m_p))     (adjoint)

``forward`` and ``adjoint`` form the phase matrix in full (M x N^2), so
they are only for tiny inputs; ``forward_points`` (a model with few nonzero
pixels) and ``adjoint_at`` (a few output pixels) evaluate the same sums for
full-size visibility sets, in chunks of visibilities.
"""

import numpy as np

from .geometry import pixel_lm


def _phase(u, v, n_img, cell):
    lm = pixel_lm(n_img, cell)
    m_grid, l_grid = np.meshgrid(lm, lm, indexing="ij")  # [iy][ix]
    return -2.0 * np.pi * (np.outer(u, l_grid.ravel()) + np.outer(v, m_grid.ravel()))


def forward(image, u, v, cell):
    """Visibilities of an N x N image (complex or real) at (u, v)."""
    n = image.shape[0]
    e = np.exp(1j * _phase(u, v, n, cell))
    return e @ np.asarray(image, dtype=np.complex128).ravel()


def adjoint(vis, u, v, cell, n_img):
    """Adjoint of ``forward``: an N x N complex image."""
    e = np.exp(-1j * _phase(u, v, n_img, cell))
    return (np.asarray(vis, dtype=np.complex128) @ e).reshape(n_img, n_img)


def forward_points(amp, iy, ix, u, v, cell, n_img):
    """A x for the model x with x[iy[j], ix[j]] = amp[j] (zero elsewhere)."""
    lm = pixel_lm(n_img, cell)
    l0, m0 = lm[np.asarray(ix)], lm[np.asarray(iy)]
    ph = -2.0 * np.pi * (np.outer(u, l0) + np.outer(v, m0))
    return np.exp(1j * ph) @ np.asarray(amp, dtype=np.complex128)


def adjoint_at(vis, u, v, cell, n_img, iy, ix, chunk=1 << 20):
    """(A^H vis) at the pixels (iy[j], ix[j]); sums over the visibilities in
    chunks of ``chunk`` (in the order of the visibilities)."""
    lm = pixel_lm(n_img, cell)
    l0, m0 = lm[np.asarray(ix)], lm[np.asarray(iy)]
    vis = np.asarray(vis, dtype=np.complex128)
    out = np.zeros(len(l0), np.complex128)
    for b in range(0, len(vis), chunk):
        e = slice(b, b + chunk)
        ph = 2.0 * np.pi * (np.outer(u[e], l0) + np.outer(v[e], m0))
        out += vis[e] @ np.exp(1j * ph)
    return out
