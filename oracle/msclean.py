"""Multi-scale CLEAN minor cycle (Eq. 6 and Eq. 7, Section 4.2) in FP64.

The paper uses the multi-scale CLEAN of Cornwell (2008) through RASCIL and
gives only its inputs: the residual (dirty) image, the PSF H, the scale set
S and the iteration cap K, plus a gain-free threshold (Section 5.1).  The
steps below are the algorithm as that reference describes it, with the
readings the paper leaves open stated where they are taken:

1.  Scale functions phi_s (``scale_kernel``): phi_0 is a unit impulse; for
    s > 0 a truncated paraboloid 1 - (r/s)^2 on r < s, normalised to unit
    sum (reading: no spheroidal taper).
2.  Smoothed residuals R_s = phi_s * R and cross PSFs B_st = phi_s * phi_t *
    psf2, linear convolutions cropped to the input's own grid ("same").
3.  Each iteration: peak (s*, p*) = argmax over the active scales of
    bias_s |R_s(p)| with bias_s = 1 - 0.6 s / s_max (reading); ties go to
    the smaller scale, then the smaller flat index iy * N + ix.
4.  Stop before the iteration if max |R_0| < threshold, R_0 the unsmoothed
    residual (reading: the threshold is on the residual image, in its own
    units), or after K iterations.
5.  alpha = gain * R_{s*}(p*) / B_{s* s*}(0); the model gets alpha phi_{s*}
    centred at p*; every R_t loses alpha B_{s* t} shifted to p*.

The PSF is the 2N x 2N image of imaging.psf2 (centre (N, N)), so a unit
source at pixel q of the N x N image contributes psf2[N + p - q] at p.

Parity: pinned by the Hogbom reduction, the single-source closed form, the
consistency R_0 = dirty - psf * model, flux conservation, and the
invariant R_t = phi_t * R_0 on pixels at least the kernel radius from the
edge, which holds only if every cross PSF B_st and every R_t update is
right (tests).  ``scale_subset`` (psi^1 of Eq. 7) is a reading of a rule
the paper states only in words: parity unpinned.
"""

import numpy as np
from scipy import signal


def scale_kernel(s):
    """phi_s on a (2r+1)^2 grid, r = ceil(s) - 1 for s > 0; unit sum."""
    if s == 0:
        return np.ones((1, 1))
    r = int(np.ceil(s)) - 1
    y, x = np.mgrid[-r:r + 1, -r:r + 1].astype(np.float64)
    k = 1.0 - (x * x + y * y) / float(s * s)
    k[k < 0.0] = 0.0
    return k / k.sum()


def convolve_same(img, kern):
    """Linear convolution of img by an odd-sized kernel, cropped to img's
    grid (zero outside the image)."""
    if kern.shape == (1, 1):
        return np.asarray(img, np.float64) * kern[0, 0]
    return signal.convolve2d(np.asarray(img, np.float64), kern, mode="same")


def scale_bias(scales, slope=0.6):
    """bias_s = 1 - slope * s / s_max (1 everywhere if s_max = 0)."""
    smax = max(scales)
    if smax == 0:
        return [1.0 for _ in scales]
    return [1.0 - slope * s / smax for s in scales]


def cross_psfs(psf2, scales):
    """B[(a, b)] = phi_a * phi_b * psf2 for scale indices a <= b."""
    ker = [scale_kernel(s) for s in scales]
    out = {}
    for a in range(len(scales)):
        for b in range(a, len(scales)):
            ab = signal.convolve2d(ker[a], ker[b], mode="full")
            out[(a, b)] = convolve_same(psf2, ab)
    return out


def add_component(model, kern, iy, ix, amp):
    """model += amp * kern centred at (iy, ix), clipped to the image."""
    n = model.shape[0]
    r = kern.shape[0] // 2
    for dy in range(-r, r + 1):
        y = iy + dy
        if y < 0 or y >= n:
            continue
        for dx in range(-r, r + 1):
            x = ix + dx
            if 0 <= x < n:
                model[y, x] += amp * kern[dy + r, dx + r]


def msclean(dirty, psf2, scales, gain=0.1, niter=2000, threshold=0.0, active=None,
            bias_slope=0.6, state=None):
    """Run the minor cycle.  Returns (model, residual R_0, components) with
    components a list of (scale index, iy, ix, alpha) in iteration order.

    ``scales`` is the scale list S in pixels; ``active`` (optional) the
    indices of S the peak search may pick (psi^n of Eq. 7); scale 0 need not
    be in S - the unsmoothed residual R_0 is tracked for the threshold
    anyway.

    ``state`` (optional dict) receives, without changing any result:
    "resid", the smoothed residuals R_t after the last iteration, and
    "gaps", per iteration the margin between the chosen candidate's biased
    value and the best value of every other (scale, pixel) candidate (a
    margin near zero marks a near-tie that rounding could reorder).
    """
    dirty = np.asarray(dirty, np.float64)
    psf2 = np.asarray(psf2, np.float64)
    n = dirty.shape[0]
    scales = list(scales)
    active = list(range(len(scales))) if active is None else list(active)
    bias = scale_bias(scales, bias_slope)
    kern = [scale_kernel(s) for s in scales]
    resid = [convolve_same(dirty, k) for k in kern]
    r0 = dirty.copy()
    cross = cross_psfs(psf2, scales)
    psf_plain = [convolve_same(psf2, k) for k in kern]  # phi_t * psf2 for the R_0 update
    model = np.zeros((n, n))
    comps = []
    gaps = []
    for _ in range(niter):
        if np.abs(r0).max() < threshold:
            break
        best_v, best_s, best_p = -1.0, -1, -1
        for si in active:  # increasing scale index: ties keep the smaller scale
            v = bias[si] * np.abs(resid[si])
            p = int(np.argmax(v))  # first occurrence: smallest flat index
            if v.flat[p] > best_v:
                best_v, best_s, best_p = v.flat[p], si, p
        if state is not None:
            second = -1.0
            for si in active:
                v = (bias[si] * np.abs(resid[si])).ravel()
                if si == best_s:
                    if v.size > 1:
                        second = max(second, np.partition(v, -2)[-2])
                else:
                    second = max(second, v.max())
            gaps.append(best_v - second)
        iy, ix = divmod(best_p, n)
        b_ss = cross[(best_s, best_s)]
        alpha = gain * resid[best_s][iy, ix] / b_ss[n, n]
        add_component(model, kern[best_s], iy, ix, alpha)
        win = (slice(n - iy, 2 * n - iy), slice(n - ix, 2 * n - ix))
        for t in range(len(scales)):
            b = cross[(min(best_s, t), max(best_s, t))]
            resid[t] -= alpha * b[win]
        r0 -= alpha * psf_plain[best_s][win]
        comps.append((best_s, iy, ix, alpha))
    if state is not None:
        state["resid"] = resid
        state["gaps"] = gaps
    return model, r0, comps


def scale_subset(scales, n_img, ell, delta, node):
    """psi^1 of Eq. 7: the scales present in the node's own domain at the
    first major cycle (reading; parity unpinned): V_L keeps s >= N / (2 (ell + delta)),
    V_H keeps s <= N / (ell - delta); if none qualifies, the scale of S
    nearest to the bound.  Returns indices into ``scales``."""
    scales = list(scales)
    if node == "L":
        bound = n_img / (2.0 * (ell + delta))
        idx = [i for i, s in enumerate(scales) if s >= bound]
    else:
        bound = n_img / (ell - delta)
        idx = [i for i, s in enumerate(scales) if s <= bound]
    if not idx:
        idx = [int(np.argmin([abs(s - bound) for s in scales]))]
    return idx
