"""Decentralized pieces around the measurement operator, in FP64:
filters Gamma, the pseudo-full-resolution composition of Eq. 7, the
aggregate rho and exchanged Phi of Eqs. 5 and 7, and the final combination.

Node names: ``own`` is the node doing the work (V_L or V_H), ``other`` the
node whose filtered deconvolved residuals it receives.

Parity unpinned (the paper gives no formula, so only the reading is
implemented): the shape of the Gamma ramp (``gamma_low``) and the values of
gamma and mu (``weights_schedule``); the pins fix where they enter Eqs. 5
and 7.
"""

import numpy as np

from .imaging import apply_psf


def gamma_low(n, ell, delta, scale=1.0):
    """Gamma_L on an n x n DFT grid in numpy FFT ordering.

    Section 4.1 asks the filters to keep only their own spatial frequencies
    and to have weights summing to one on the overlap L n H.  Reading
    (shape parity unpinned): a radial linear ramp
        Gamma_L(kappa) = clip((ell + delta - kappa) / (2 delta), 0, 1)
    with kappa the radius of the DFT frequency in Fourier pixels of the
    N x N image; for a 2N x 2N image the same physical frequency has twice
    the index, so ``scale`` = 2 there.
    """
    k = np.fft.fftfreq(n, d=1.0 / n)
    ky, kx = np.meshgrid(k, k, indexing="ij")
    kappa = np.sqrt(kx * kx + ky * ky) / scale
    return np.clip((ell + delta - kappa) / (2.0 * delta), 0.0, 1.0)


def gamma_high(n, ell, delta, scale=1.0):
    """Gamma_H = 1 - Gamma_L, so Gamma_L + Gamma_H is the identity."""
    return 1.0 - gamma_low(n, ell, delta, scale)


def apply_filter(img, filt):
    """Gamma x = Re F^-1 (Gamma . F x) on the image's own periodic grid."""
    return np.fft.ifft2(np.fft.fft2(img) * filt).real


def filters(n_img, ell, delta, own):
    """(Gamma_own, Gamma_other) for an N x N image; own in {'L', 'H'}."""
    lo = gamma_low(n_img, ell, delta)
    return (lo, 1.0 - lo) if own == "L" else (1.0 - lo, lo)


def psf_filters(n_img, ell, delta, own):
    """Same as ``filters`` for the 2N x 2N PSF grid."""
    lo = gamma_low(2 * n_img, ell, delta, scale=2.0)
    return (lo, 1.0 - lo) if own == "L" else (1.0 - lo, lo)


def weights_schedule(cycle, w_own, w_other):
    """(gamma^n, mu^n) of Eq. 7.

    Section 4.2 fixes gamma = 1, mu = 0 at the first major cycle and calls
    them, afterwards, weights that re-normalise the PSF and dirty images
    globally (each is first normalised by its local visibilities).  Reading:
    gamma = W_own / (W_own + W_other), mu = W_other / (W_own + W_other),
    with W the summed imaging weights of each partition (parity unpinned).
    """
    if cycle <= 1:
        return 1.0, 0.0
    tot = w_own + w_other
    return w_own / tot, w_other / tot


def compose_dirty(resid_own, rho_other, psf_other, ell, delta, own, gamma, mu):
    """Eq. 7 dirty image: gamma Gamma_own i~_own + mu H_other rho_other."""
    g_own, _ = filters(resid_own.shape[0], ell, delta, own)
    out = gamma * apply_filter(resid_own, g_own)
    if mu != 0.0 and rho_other is not None:
        out = out + mu * apply_psf(psf_other, rho_other)
    return out


def compose_psf(psf_own, psf_other, ell, delta, own, gamma, mu):
    """Eq. 7 PSF: gamma Gamma_own H_own + mu Gamma_other H_other (2N x 2N)."""
    n = psf_own.shape[0] // 2
    g_own, g_other = psf_filters(n, ell, delta, own)
    out = gamma * apply_filter(psf_own, g_own)
    if mu != 0.0:
        out = out + mu * apply_filter(psf_other, g_other)
    return out


def exchange(delta_own, ell, delta, own):
    """Phi sent to the other node after a major cycle (Eq. 5 and Eq. 7):
    Gamma_own applied to the node's latest deconvolved residual."""
    g_own, _ = filters(delta_own.shape[0], ell, delta, own)
    return apply_filter(delta_own, g_own)


def update_rho(rho_other, phi_received, delta_own, ell, delta, own):
    """Aggregate update (Section 4.1): add the received Phi and subtract the
    other node's filter applied to the local deconvolved residual,
        rho^n = rho^{n-1} + Phi^n - Gamma_other ibar_own^n."""
    _, g_other = filters(delta_own.shape[0], ell, delta, own)
    prev = np.zeros_like(delta_own) if rho_other is None else rho_other
    return prev + phi_received - apply_filter(delta_own, g_other)


def combine(images, weights=None):
    """Final image: weighted average of the nodes' images; the paper uses
    equal weights 0.5 / 0.5 (Section 5.2)."""
    if weights is None:
        weights = [1.0 / len(images)] * len(images)
    out = np.zeros_like(np.asarray(images[0], np.float64))
    for w, im in zip(weights, images):
        out = out + w * np.asarray(im, np.float64)
    return out


def reconstruct_msclean(u, v, vis, w, n_img, cell, n_cycles, scales, gain=0.1, niter=2000,
                        threshold=0.0, partitions=2, ell=None, delta=1.0, support=8,
                        record_gaps=False, workers=None, minor=None):
    """The major/minor loop with multi-scale CLEAN, serial (partitions = 1)
    or decentralized over V_L / V_H (partitions = 2), in FP64.

    Per major cycle n and node (Section 4.2):
      i~     = residual of the node's own model on its own visibilities (Eq. 2)
      D, P   = gamma Gamma_own i~ + mu H_other rho_other,
               gamma Gamma_own H_own + mu Gamma_other H_other           (Eq. 7)
      ibar   = ms-CLEAN(D, P, psi^n, K), psi^1 the node's own scales    (Eq. 7)
      model += ibar                                                     (Eq. 3)
    then the nodes exchange Phi = Gamma_own ibar and update rho (Section
    4.1); the final image is the equal-weight average (Section 5.2).
    Serially the loop is Eq. 2 -> ms-CLEAN(i~, H, S, K) -> Eq. 3.

    Returns (final image, per-node models, history) with history a list of
    per-cycle dicts {node: (dirty D, psf P, components, ibar, gaps)}; gaps
    is the per-iteration near-tie margin of ``msclean.msclean`` with
    ``record_gaps``, else None.

    ``workers`` (optional) runs the residuals and PSFs on that many host
    processes (``pool``: the same operators, with the FP64 additions of the
    grid cells in chunk order).  ``minor`` (optional) replaces the minor
    cycle: minor(cycle, node, D, P, active) -> (ibar, components, gaps),
    for running the loop on another precision's inputs or replaying a
    recorded run.
    """
    from . import imaging, msclean as msc
    if workers is not None:
        from . import pool
    m = len(u)
    if partitions == 1:
        masks = {"L": np.ones(m, bool)}
        nodes = ("L",)
    else:
        low, high, ell = imaging.partition(u, v, n_img, cell, ell=ell, delta=delta)
        masks = {"L": low, "H": high}
        nodes = ("L", "H")
    other = {"L": "H", "H": "L"}
    if workers is None:
        psf = {k: imaging.psf2(u[mk], v[mk], w[mk], n_img, cell, support=support)
               for k, mk in masks.items()}
    else:
        psf = {k: pool.psf2(u[mk], v[mk], w[mk], n_img, cell, support=support, workers=workers)
               for k, mk in masks.items()}
    wsum = {k: w[mk].sum() for k, mk in masks.items()}
    models = {k: np.zeros((n_img, n_img)) for k in nodes}
    rho = {k: np.zeros((n_img, n_img)) for k in nodes}   # rho_other held by node k
    history = []
    for cyc in range(1, n_cycles + 1):
        step, deltas = {}, {}
        for k in nodes:
            mk = masks[k]
            if workers is None:
                resid, _ = imaging.residual_image(u[mk], v[mk], vis[mk], w[mk], models[k], cell,
                                                  support=support)
            else:
                resid, _ = pool.residual_image(u[mk], v[mk], vis[mk], w[mk], models[k], cell,
                                               support=support, workers=workers)
            if partitions == 1:
                d_img, p_img, active = resid, psf[k], None
            else:
                gamma, mu = weights_schedule(cyc, wsum[k], wsum[other[k]])
                d_img = compose_dirty(resid, rho[k], psf[other[k]], ell, delta, k, gamma, mu)
                p_img = compose_psf(psf[k], psf[other[k]], ell, delta, k, gamma, mu)
                active = msc.scale_subset(scales, n_img, ell, delta, k) if cyc == 1 else None
            if minor is not None:
                ibar, comps, gaps = minor(cyc, k, d_img, p_img, active)
            else:
                st = {} if record_gaps else None
                ibar, _, comps = msc.msclean(d_img, p_img, scales, gain, niter, threshold,
                                             active, state=st)
                gaps = st["gaps"] if record_gaps else None
            deltas[k] = ibar
            step[k] = (d_img, p_img, comps, ibar, gaps)
        for k in nodes:
            models[k] = models[k] + deltas[k]
        if partitions == 2:
            new_rho = {}
            for k in nodes:
                phi_recv = exchange(deltas[other[k]], ell, delta, other[k])
                new_rho[k] = update_rho(rho[k], phi_recv, deltas[k], ell, delta, k)
            rho = new_rho
        history.append(step)
    final = combine([models[k] for k in nodes])
    return final, models, history


def reconstruct_fista(u, v, vis, w, n_img, cell, n_cycles, start_images, lam_frac=1e-3,
                      n_iter=200, power_iters=30, vanishing=8, levels=3, partitions=2, ell=None,
                      delta=1.0, support=8, dictionary=False, workers=None):
    """The major/minor loop with the sparsity-regularised minor cycle (Eqs.
    4 and 5), serial (partitions = 1) or decentralized, in FP64.

    Per major cycle n and node: i~ = the node's residual (Eq. 2); lambda^n =
    lam_frac max |i~| (reading of "1e-3 x max |dirty|"); gamma_n = 0 at
    n = 1, else 1 (Eq. 5); L_hat by ``power_iters`` power iterations from
    start_images[node]; alpha by ``n_iter`` FISTA iterations; ibar = W alpha
    (W one db_vanishing basis, or with ``dictionary`` the tight frame of db1 ..
    db_vanishing);
    model += ibar (Eq. 3).  Then the Phi / rho exchange of Section 4.1 and,
    at the end, the equal-weight combination of Section 5.2.
    Returns (final image, per-node models, history of per-cycle dicts
    {node: (lambda, L_hat, objective list)}).  ``workers`` as in
    ``reconstruct_msclean``.
    """
    from . import fista as fs, imaging, wavelets
    if workers is not None:
        from . import pool
    # one Daubechies basis, or the concatenation of the first `vanishing` ones
    h = ([wavelets.daubechies(p) for p in range(1, vanishing + 1)] if dictionary
         else wavelets.daubechies(vanishing))
    m = len(u)
    if partitions == 1:
        masks = {"L": np.ones(m, bool)}
        nodes = ("L",)
    else:
        low, high, ell = imaging.partition(u, v, n_img, cell, ell=ell, delta=delta)
        masks = {"L": low, "H": high}
        nodes = ("L", "H")
    other = {"L": "H", "H": "L"}
    if workers is None:
        psf = {k: imaging.psf2(u[mk], v[mk], w[mk], n_img, cell, support=support)
               for k, mk in masks.items()}
    else:
        psf = {k: pool.psf2(u[mk], v[mk], w[mk], n_img, cell, support=support, workers=workers)
               for k, mk in masks.items()}
    models = {k: np.zeros((n_img, n_img)) for k in nodes}
    rho = {k: np.zeros((n_img, n_img)) for k in nodes}
    history = []
    for cyc in range(1, n_cycles + 1):
        step, deltas = {}, {}
        for k in nodes:
            mk = masks[k]
            if workers is None:
                resid, _ = imaging.residual_image(u[mk], v[mk], vis[mk], w[mk], models[k], cell,
                                                  support=support)
            else:
                resid, _ = pool.residual_image(u[mk], v[mk], vis[mk], w[mk], models[k], cell,
                                               support=support, workers=workers)
            gamma_n = 0.0 if (cyc == 1 or partitions == 1) else 1.0
            lam = lam_frac * float(np.abs(resid).max())
            prob = fs.NodeProblem(resid, psf[k], rho[k], gamma_n, ell, delta, k, h, levels,
                                  serial=(partitions == 1))
            L_hat = fs.power_iteration(prob, start_images[k], power_iters)
            alpha, obj = fs.fista(prob, lam, n_iter, L_hat)
            deltas[k] = prob.W(alpha)
            step[k] = (lam, L_hat, obj)
        for k in nodes:
            models[k] = models[k] + deltas[k]
        if partitions == 2:
            rho = {k: update_rho(rho[k], exchange(deltas[other[k]], ell, delta, other[k]),
                                 deltas[k], ell, delta, k) for k in nodes}
        history.append(step)
    return combine([models[k] for k in nodes]), models, history
