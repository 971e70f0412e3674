"""FISTA for the sparsity-regularised minor cycle (Eqs. 4 and 5, Section
4.1), in FP64.

For node ``own`` of the decentralized problem (Eq. 5; the serial Eq. 4 is
the special case with Gamma_own = I and gamma_n = 0):

    f(alpha) = || Gamma_own (i~ - H W alpha) ||^2 + gamma_n || rho - Gamma_other W alpha ||^2
    alpha*   = argmin f(alpha) + lambda ||alpha||_1,     ibar = W alpha*

with W the orthonormal periodized wavelet synthesis (``wavelets.idwt2``)
or, for a list of filters, the tight frame of their concatenation
(``wavelets.dict_synthesis``: the paper's first-8-Daubechies dictionary),
H the convolution by the node's 2N x 2N PSF (``imaging.apply_psf``) and
the filters Gamma of ``decentral``.  H and Gamma are self-adjoint (reading:
the PSF is even and the filters are real and radial), so

    grad f = -2 W^T [ H Gamma_own^2 (i~ - H W alpha) + gamma_n Gamma_other (rho - Gamma_other W alpha) ].

FISTA (Beck and Teboulle 2009) with constant step 1/L_hat:
    alpha_k = soft(y_k - grad f(y_k) / L_hat, lambda / L_hat)
    t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2
    y_{k+1} = alpha_k + ((t_k - 1) / t_{k+1}) (alpha_k - alpha_{k-1})
from alpha_0 = y_1 = 0, t_1 = 1.  L_hat = 2 lambda_max of the image-space
map x -> H Gamma_own^2 H x + gamma_n Gamma_other^2 x (W is orthonormal),
estimated by power iteration from a given start image (the random start
is an input, so both implementations can use the same one).  For the tight
frame W^T M W has the nonzero eigenvalues of M W W^T = M, so the same
image-space estimate applies.
"""

import numpy as np

from . import decentral, wavelets
from .imaging import apply_psf


def soft(x, t):
    """Soft thresholding sign(x) max(|x| - t, 0)."""
    return np.sign(x) * np.maximum(np.abs(x) - t, 0.0)


class NodeProblem:
    """Operators of Eq. 5 for one node (or Eq. 4 when serial)."""

    def __init__(self, dirty, psf2, rho, gamma_n, ell, delta, own, h, levels, serial=False):
        self.dirty = np.asarray(dirty, np.float64)
        self.psf = np.asarray(psf2, np.float64)
        self.rho = None if rho is None else np.asarray(rho, np.float64)
        self.gamma_n = float(gamma_n)
        self.h, self.levels = h, levels
        n = self.dirty.shape[0]
        if serial:
            self.g_own, self.g_other = np.ones((n, n)), np.zeros((n, n))
        else:
            self.g_own, self.g_other = decentral.filters(n, ell, delta, own)

    def W(self, a):
        if isinstance(self.h, list):
            return wavelets.dict_synthesis(a, self.h, self.levels)
        return wavelets.idwt2(a, self.h, self.levels)

    def Wt(self, x):
        if isinstance(self.h, list):
            return wavelets.dict_analysis(x, self.h, self.levels)
        return wavelets.dwt2(x, self.h, self.levels)

    def gam(self, x, g):
        return decentral.apply_filter(x, g)

    def normal_map(self, x):
        """x -> H Gamma_own^2 H x + gamma_n Gamma_other^2 x (image space)."""
        out = apply_psf(self.psf, self.gam(self.gam(apply_psf(self.psf, x), self.g_own), self.g_own))
        if self.gamma_n != 0.0:
            out = out + self.gamma_n * self.gam(self.gam(x, self.g_other), self.g_other)
        return out

    def objective(self, a, lam):
        x = self.W(a)
        r1 = self.gam(self.dirty - apply_psf(self.psf, x), self.g_own)
        f = float(np.sum(r1 * r1))
        if self.gamma_n != 0.0:
            r2 = self.rho - self.gam(x, self.g_other)
            f += self.gamma_n * float(np.sum(r2 * r2))
        return f + lam * float(np.abs(a).sum())

    def grad(self, a):
        x = self.W(a)
        t = apply_psf(self.psf, self.gam(self.gam(self.dirty - apply_psf(self.psf, x),
                                                  self.g_own), self.g_own))
        if self.gamma_n != 0.0:
            t = t + self.gamma_n * self.gam(self.rho - self.gam(x, self.g_other), self.g_other)
        return -2.0 * self.Wt(t)


def power_iteration(prob, start, iters=30):
    """2 lambda_max of the normal map by power iteration from ``start``."""
    x = np.asarray(start, np.float64)
    x = x / np.linalg.norm(x)
    lam = 0.0
    for _ in range(iters):
        y = prob.normal_map(x)
        lam = float(np.linalg.norm(y))
        x = y / lam
    return 2.0 * lam


def fista(prob, lam, n_iter, L_hat):
    """Returns (alpha, objective per iteration)."""
    a_prev = np.zeros(prob.Wt(np.zeros(prob.dirty.shape)).shape)
    y = a_prev.copy()
    t = 1.0
    obj = []
    for _ in range(n_iter):
        a = soft(y - prob.grad(y) / L_hat, lam / L_hat)
        t_next = (1.0 + np.sqrt(1.0 + 4.0 * t * t)) / 2.0
        y = a + ((t - 1.0) / t_next) * (a - a_prev)
        a_prev, t = a, t_next
        obj.append(prob.objective(a, lam))
    return a_prev, obj
