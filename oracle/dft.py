"""Direct Fourier sums: the plain definition of the measurement operator.

Eq. 1 (Section 2) with the direction-independent and direction-dependent
terms set to one and the w term dropped reduces, as Section 2 states, to a
two-dimensional Fourier transform.  Reading: the 1/n factor is
dropped too, and the sky is the pixelised model image, so

    (A x)_k  = sum_p x_p exp(-2 pi i (u_k l_p + v_k m_p))      (forward)
    (A^H y)_p = sum_k y_k exp(+2 pi i (u_k l_p + v_k m_p))     (adjoint)

The phase matrix is formed in full (M x N^2), so this module is only for
tiny inputs.
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
