"""Coordinate chain shared by every operator of the oracle.

The paper states the measurement equation (Eq. 1, Section 2) in terms of
baseline coordinates (u, v, w) in wavelengths and direction cosines (l, m);
it gives no pixel or grid convention.  The conventions below are readings
and are applied identically by the GPU library:

* image of N x N pixels, row-major ``[iy][ix]``, pixel (ix, iy) at
  l = (ix - N/2) * cell, m = (iy - N/2) * cell; the phase centre is pixel
  (N/2, N/2);
* u_lambda = uvw_metres * (freq / c): one multiplication by a host-side
  FP64 constant, so both implementations round identically;
* grid of Ng = sigma * N cells with spacing du = 1 / (Ng * cell); the grid
  coordinate of a visibility is x = u_lambda * (Ng * cell) + Ng / 2 (cell
  centres sit at integers), multiplication then addition, no fused
  multiply-add;
* "Fourier pixels" of the N x N image (the unit of the partition radius ell
  and delta, Table 2 and Section 5.1) are u_lambda * (N * cell).
"""

import numpy as np

C_LIGHT = 299792458.0


def wavelength_scale(freq_hz):
    """FP64 factor turning metres into wavelengths."""
    return np.float64(freq_hz) / np.float64(C_LIGHT)


def uv_lambda(uvw_m, freq_hz):
    """(u, v) in wavelengths for baseline coordinates in metres [M, 3]."""
    s = wavelength_scale(freq_hz)
    uvw_m = np.asarray(uvw_m, dtype=np.float64)
    return uvw_m[:, 0] * s, uvw_m[:, 1] * s


def grid_coord(u_lam, n_grid, cell):
    """Grid coordinate in cells: u * (Ng * cell) + Ng / 2."""
    scale = np.float64(n_grid) * np.float64(cell)
    return np.asarray(u_lam, np.float64) * scale + np.float64(n_grid // 2)


def fourier_pixels(u_lam, n_img, cell):
    """u in Fourier pixels of the N x N image: u * (N * cell)."""
    return np.asarray(u_lam, np.float64) * (np.float64(n_img) * np.float64(cell))


def default_cell(u_lam, v_lam):
    """Pixel size used by the synthetic workloads and by cell=0:
    1 / (3 * max(|u|, |v|)), so the sampled uv extent covers two thirds of
    the half-width of a 2x padded grid and the kernel halo never wraps."""
    return 1.0 / (3.0 * max(np.max(np.abs(u_lam)), np.max(np.abs(v_lam))))


def pixel_lm(n_img, cell):
    """Direction cosine of each pixel index along one axis."""
    return (np.arange(n_img, dtype=np.float64) - n_img // 2) * np.float64(cell)
