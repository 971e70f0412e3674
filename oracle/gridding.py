"""Kernel-based (gridded) measurement operator in FP64.

This is the same algorithm the GPU library runs, written as the composition
of its plain steps with no blocking or fusion:

    A_G   = K  . F_c  . P   . diag(1 / psi_hat (x) psi_hat)
    A_G^H = diag(1 / psi_hat (x) psi_hat) . P^T . F_c^H . K^T

* diag(1/psi_hat): gridding correction (es_kernel.correction), separable
  over the two image axes;
* P: zero-padding of the N x N image into the centre of the Ng x Ng image
  (pixel ix goes to ix + (Ng - N)/2);
* F_c: centred unnormalised 2-D DFT,
      F_c[g] = sum_j x[j] exp(-2 pi i (g - Ng/2)(j - Ng/2) / Ng)  per axis,
  so grid cell g holds spatial frequency (g - Ng/2) * du; F_c^H uses +i;
* K: degridding - each visibility is the sum over its W x W tap cells of
  phi_x * phi_y * grid (cell indices taken modulo Ng); K^T is gridding.

Section 2 writes the residual as F^dagger G (v - G^dagger F i_hat) (Eq. 2)
with G, G^dagger the gridding and degridding operators; in the notation
above G^dagger F = A_G and F^dagger G = A_G^H.  The correction and padding
belong to the gridder the paper uses (Section 2 cites the improved
w-gridder); they are what makes A_G approximate the direct sum of ``dft``.
"""

import numpy as np

from .es_kernel import correction, taps


def centred_fft2(x):
    """F_c along both axes (unnormalised)."""
    return np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(x)))


def centred_ifft2(y):
    """F_c^H along both axes (unnormalised, so F_c^H F_c = Ng^2 I)."""
    return np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(y))) * y.size


def pad_centre(img, n_grid):
    n = img.shape[0]
    out = np.zeros((n_grid, n_grid), dtype=np.complex128)
    o = (n_grid - n) // 2
    out[o:o + n, o:o + n] = img
    return out


def crop_centre(grid_img, n_img):
    o = (grid_img.shape[0] - n_img) // 2
    return grid_img[o:o + n_img, o:o + n_img]


def degrid(grid, gx, gy, support, beta):
    """K: visibilities at grid coordinates (gx, gy) from an Ng x Ng grid."""
    ng = grid.shape[0]
    fx, wx = taps(gx, support, beta)
    fy, wy = taps(gy, support, beta)
    out = np.zeros(gx.shape, dtype=np.complex128)
    for j in range(support):
        row = (fy + j) % ng
        for i in range(support):
            col = (fx + i) % ng
            out += wy[:, j] * wx[:, i] * grid[row, col]
    return out


def grid_vis(vis, gx, gy, n_grid, support, beta, block=1 << 18):
    """K^T: accumulate visibilities onto an Ng x Ng grid.

    Every (visibility, tap) pair adds vis_k * wy_k[j] * wx_k[i] to cell
    ((fy_k + j) mod Ng, (fx_k + i) mod Ng); the pairs of ``block``
    visibilities at a time are summed by one bincount (FP64)."""
    fx, wx = taps(gx, support, beta)
    fy, wy = taps(gy, support, beta)
    vis = np.asarray(vis, dtype=np.complex128)
    acc_re = np.zeros(n_grid * n_grid)
    acc_im = np.zeros(n_grid * n_grid)
    t = np.arange(support)
    for a in range(0, len(vis), block):
        e = slice(a, a + block)
        rows = (fy[e, None] + t) % n_grid                          # [m, W]
        cols = (fx[e, None] + t) % n_grid                          # [m, W]
        flat = (rows[:, :, None] * n_grid + cols[:, None, :]).ravel()  # [m, W, W]
        w = wy[e, :, None] * wx[e, None, :]                        # [m, W, W]
        acc_re += np.bincount(flat, weights=(w * vis[e].real[:, None, None]).ravel(),
                              minlength=n_grid * n_grid)
        acc_im += np.bincount(flat, weights=(w * vis[e].imag[:, None, None]).ravel(),
                              minlength=n_grid * n_grid)
    return (acc_re + 1j * acc_im).reshape(n_grid, n_grid)


def forward(image, gx, gy, n_grid, support, beta):
    """A_G x: predicted visibilities of an N x N image."""
    n = image.shape[0]
    psi = correction(n, n_grid, support, beta)
    corrected = np.asarray(image, dtype=np.complex128) / np.outer(psi, psi)
    return degrid(centred_fft2(pad_centre(corrected, n_grid)), gx, gy, support, beta)


def adjoint(vis, gx, gy, n_img, n_grid, support, beta):
    """A_G^H y: an N x N complex image."""
    psi = correction(n_img, n_grid, support, beta)
    g = grid_vis(vis, gx, gy, n_grid, support, beta)
    return crop_centre(centred_ifft2(g), n_img) / np.outer(psi, psi)
