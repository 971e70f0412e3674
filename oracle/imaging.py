"""Weighting, spatial-frequency partition, dirty / residual images and PSF.

All quantities in FP64.  Visibility coordinates are (u, v) in wavelengths
(``geometry.uv_lambda``); ``cell`` is the pixel size in radians.
"""

import numpy as np

from . import gridding
from .es_kernel import es_beta
from .geometry import fourier_pixels, grid_coord


# --------------------------------------------------------------- weighting

def uniform_weights(u, v, n_img, cell, w_in=None, valid=None):
    """Uniform weighting (Section 5.1 images every dataset with it).

    Reading: the density cell of visibility k is the nearest
    cell of the N x N image's Fourier grid,
        c_k = (floor(u_k N cell + 0.5), floor(v_k N cell + 0.5)) mod N,
    the density is the number n(c_k) of unflagged visibilities of the whole
    data set in that cell (counted before any partition, so serial and
    decentralized runs share weights), and w_k = w_in_k / n(c_k).  With
    equal input weights this is the textbook uniform weighting.  Flagged
    visibilities get weight 0.
    """
    m = len(u)
    w_in = np.ones(m) if w_in is None else np.asarray(w_in, np.float64)
    valid = np.ones(m, bool) if valid is None else np.asarray(valid, bool)
    cu = np.floor(fourier_pixels(u, n_img, cell) + 0.5).astype(np.int64) % n_img
    cv = np.floor(fourier_pixels(v, n_img, cell) + 0.5).astype(np.int64) % n_img
    key = cv * n_img + cu
    counts = np.bincount(key[valid], minlength=n_img * n_img)
    w = np.zeros(m)
    w[valid] = w_in[valid] / counts[key[valid]]
    return w


# --------------------------------------------------------------- partition

def radius_pixels(u, v, n_img, cell):
    """rho_k = |(u_k, v_k)| in Fourier pixels of the N x N image (the unit of
    ell in Table 2): sqrt(pu^2 + pv^2) with pu = u * (N cell)."""
    pu = fourier_pixels(u, n_img, cell)
    pv = fourier_pixels(v, n_img, cell)
    return np.sqrt(pu * pu + pv * pv)


def lower_median(values):
    """Element of rank floor((n - 1) / 2) of the sorted values."""
    values = np.asarray(values, np.float64)
    k = (len(values) - 1) // 2
    return np.partition(values, k)[k]


def partition(u, v, n_img, cell, ell=None, delta=1.0, valid=None):
    """Spatial-frequency partition of Fig. 3 (Section 3).

    V_L = {rho <= ell + delta}, V_H = {rho >= ell - delta}: two overlapping
    sets whose overlap is the ring of half-width delta around the circle of
    radius ell.  delta = 1 pixel as in Section 5.1.  Reading: when ``ell``
    is None the split is at the lower median of rho over the unflagged
    visibilities (the synthetic workloads split "at the median |uv|").
    Returns (mask_L, mask_H, ell).
    """
    rho = radius_pixels(u, v, n_img, cell)
    valid = np.ones(len(u), bool) if valid is None else np.asarray(valid, bool)
    if ell is None:
        ell = lower_median(rho[valid])
    low = valid & (rho <= ell + delta)
    high = valid & (rho >= ell - delta)
    return low, high, float(ell)


# --------------------------------------------------------------- operator

class Operator:
    """The gridded operator of one visibility set at one image size.

    ``n_grid = sigma * n_img``; ``support`` W; ``beta`` defaults to 2.30 W.
    """

    def __init__(self, u, v, cell, n_img, sigma=2, support=8, beta=None):
        self.n_img = int(n_img)
        self.n_grid = int(round(sigma * n_img))
        self.support = int(support)
        self.beta = es_beta(support) if beta is None else float(beta)
        self.cell = float(cell)
        self.gx = grid_coord(u, self.n_grid, cell)
        self.gy = grid_coord(v, self.n_grid, cell)

    def forward(self, image):
        return gridding.forward(image, self.gx, self.gy, self.n_grid, self.support, self.beta)

    def adjoint(self, vis):
        return gridding.adjoint(vis, self.gx, self.gy, self.n_img, self.n_grid,
                                self.support, self.beta)


def residual_image(u, v, vis, w, model, cell, sigma=2, support=8, beta=None):
    """Eq. 2: i~ = F^dagger G (v - G^dagger F i^), as the real part of
    A_G^H (w . (v - A_G model)) normalised by sum(w).  With a zero model this
    is the dirty image.  Returns (image, predicted visibilities)."""
    n = model.shape[0]
    op = Operator(u, v, cell, n, sigma, support, beta)
    pred = op.forward(model) if np.any(model) else np.zeros(len(u), np.complex128)
    r = np.asarray(vis, np.complex128) - pred
    img = op.adjoint(np.asarray(w, np.float64) * r).real / np.sum(w)
    return img, pred


def dirty_image(u, v, vis, w, n_img, cell, sigma=2, support=8, beta=None):
    return residual_image(u, v, vis, w, np.zeros((n_img, n_img)), cell, sigma, support, beta)[0]


def psf2(u, v, w, n_img, cell, sigma=2, support=8, beta=None, normalise=True):
    """PSF on a 2N x 2N image with the same pixel size: Re A'^H(w) / sum(w)
    (peak sum(w) before normalisation).  Reading: the paper uses the PSF as
    the surrogate of the measurement operator (H in Eqs. 4, 5 and 7) without
    stating its size; 2N makes H equal to the normal operator on N x N
    images.  Its centre is pixel (N, N)."""
    op = Operator(u, v, cell, 2 * n_img, sigma, support, beta)
    img = op.adjoint(np.asarray(w, np.float64)).real
    return img / np.sum(w) if normalise else img


def apply_psf(psf, x):
    """H x for an N x N image x and a 2N x 2N PSF centred at (N, N):
        (H x)(p) = sum_q psf[N + p - q] x(q),
    a plain linear convolution evaluated with scipy.signal.fftconvolve."""
    from scipy.signal import fftconvolve
    n = x.shape[0]
    full = fftconvolve(psf, x, mode="full")  # index (a + b) of psf[a] x[b]
    return full[n:2 * n, n:2 * n]
