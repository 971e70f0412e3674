"""Orthonormal Daubechies wavelets and the periodized 2-D transform W, FP64.

The sparsity-regularised reconstruction (Section 4.1, Eqs. 4 and 5) uses a
wavelet operator W; the configuration read here is the
Daubechies wavelet with p = 8 vanishing moments (16 taps, extremal phase),
3 levels, periodized boundaries, with the l1 norm on every coefficient.

Filter construction (spectral factorisation, Daubechies' construction):
with y = sin^2(w/2), |m0(w)|^2 = cos^{2p}(w/2) P(y), P(y) = sum_{k<p}
C(p-1+k, k) y^k.  In the variable z = e^{iw}, y = (2 - z - 1/z)/4, so
z^{p-1} P(y(z)) is a polynomial of degree 2(p-1) whose roots come in pairs
(r, 1/conj(r)).  The filter is h(z) = sum_n h_n z^n proportional to
(1 + z)^p prod_{|r| > 1} (z - r), normalised to sum h = sqrt(2).  This
choice of one root per pair is the convention whose p = 2 member is the
classical (1 + sqrt 3, 3 + sqrt 3, 3 - sqrt 3, 1 - sqrt 3) / (4 sqrt 2)
(pinned in the tests).  Roots are polished by Newton's method in extended
precision.  The high-pass filter is g_j = (-1)^j h_{L-1-j}.

The paper's sparsity prior uses for W a concatenation of the first 8
Daubechies wavelets (Section 5.1); as a tight frame each basis is scaled
by 1/sqrt(P), P the number of bases, so that W W^T = I
(``dict_analysis`` / ``dict_synthesis``; coefficients stacked [P][n][n]).

Periodized analysis along one axis of length n (even):
    a[k] = sum_j h_j x[(2k + j) mod n],   d[k] = sum_j g_j x[(2k + j) mod n]
and synthesis is its transpose.  Coefficients are stored in place (Mallat
layout): after one 2-D level an n x n block holds [[LL, LH], [HL, HH]] with
LL (rows low, columns low) in the top-left n/2 x n/2 block, which the next
level transforms again.
"""

from math import comb

import numpy as np


def _polish(poly, root, steps=20):
    """Newton refinement of a root of poly (increasing powers) in extended precision."""
    c = np.asarray(poly, dtype=np.clongdouble)
    z = np.clongdouble(root)
    for _ in range(steps):
        p = np.clongdouble(0)
        dp = np.clongdouble(0)
        for a in c[::-1]:
            dp = dp * z + p
            p = p * z + a
        if dp == 0:
            break
        z = z - p / dp
    return z


def daubechies(p):
    """Low-pass filter h (length 2p) of the Daubechies wavelet with p
    vanishing moments (p = 1: Haar)."""
    if p == 1:
        return np.array([1.0, 1.0]) / np.sqrt(2.0)
    zy = np.array([-0.25, 0.5, -0.25])       # z * y(z), increasing powers
    poly = np.zeros(2 * p - 1)
    for k in range(p):
        t = np.array([1.0])
        for _ in range(k):
            t = np.convolve(t, zy)
        t = np.concatenate([np.zeros(p - 1 - k), t])  # times z^(p-1-k)
        poly[:len(t)] += comb(p - 1 + k, k) * t
    roots = [_polish(poly, r) for r in np.roots(poly[::-1])]
    outside = [r for r in roots if abs(r) > 1.0]
    h = np.array([1.0], dtype=np.clongdouble)
    for _ in range(p):
        h = np.convolve(h, np.array([1.0, 1.0], dtype=np.clongdouble))
    for r in outside:
        h = np.convolve(h, np.array([-r, 1.0], dtype=np.clongdouble))
    h = np.real(h)
    h = h * np.sqrt(np.longdouble(2.0)) / h.sum()
    return np.asarray(h, dtype=np.float64)


def highpass(h):
    L = len(h)
    return np.array([(-1) ** j * h[L - 1 - j] for j in range(L)])


def _analysis_axis(x, h, g, axis):
    x = np.moveaxis(np.asarray(x, np.float64), axis, -1)
    n = x.shape[-1]
    k = np.arange(n // 2)
    idx = (2 * k[:, None] + np.arange(len(h))[None, :]) % n
    a = (x[..., idx] * h).sum(-1)
    d = (x[..., idx] * g).sum(-1)
    return np.moveaxis(np.concatenate([a, d], axis=-1), -1, axis)


def _synthesis_axis(c, h, g, axis):
    c = np.moveaxis(np.asarray(c, np.float64), axis, -1)
    n = c.shape[-1]
    a, d = c[..., :n // 2], c[..., n // 2:]
    out = np.zeros(c.shape)
    for j in range(len(h)):
        pos = (2 * np.arange(n // 2) + j) % n
        np.add.at(out, (Ellipsis, pos), h[j] * a + g[j] * d)
    return np.moveaxis(out, -1, axis)


def dwt2(x, h, levels):
    """W^T: image -> coefficients (Mallat layout), periodized."""
    g = highpass(h)
    c = np.array(x, np.float64, copy=True)
    n = c.shape[0]
    for _ in range(levels):
        blk = c[:n, :n]
        blk = _analysis_axis(blk, h, g, axis=1)
        blk = _analysis_axis(blk, h, g, axis=0)
        c[:n, :n] = blk
        n //= 2
    return c


def idwt2(c, h, levels):
    """W: coefficients -> image (the inverse and adjoint of dwt2)."""
    g = highpass(h)
    x = np.array(c, np.float64, copy=True)
    n = x.shape[0] >> (levels - 1)
    for _ in range(levels):
        blk = x[:n, :n]
        blk = _synthesis_axis(blk, h, g, axis=0)
        blk = _synthesis_axis(blk, h, g, axis=1)
        x[:n, :n] = blk
        n *= 2
    return x


def dict_analysis(x, hs, levels):
    """W^T for the dictionary of bases hs: stacked coefficients, each basis
    scaled by 1 / sqrt(len(hs))."""
    k = 1.0 / np.sqrt(len(hs))
    return np.stack([k * dwt2(x, h, levels) for h in hs])


def dict_synthesis(c, hs, levels):
    """W: sum over the bases of their synthesis, scaled by 1 / sqrt(len(hs))."""
    k = 1.0 / np.sqrt(len(hs))
    out = np.zeros(c.shape[1:])
    for p, h in enumerate(hs):
        out += k * idwt2(c[p], h, levels)
    return out
