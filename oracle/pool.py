"""Runs the oracle's operators over large visibility sets on several host
processes.

Test infrastructure, like the rest of ``oracle/``.  Nothing here computes
anything the other modules do not: degridding (``gridding.degrid``) and
gridding (``gridding.grid_vis``) are called unchanged on contiguous chunks
of the visibilities in worker processes.  Degridding is per visibility, so
the chunks' outputs are concatenated; gridding is linear in the
visibilities, so the chunks' grids are added, in chunk order, in FP64.
The only difference from one serial call is the order of the FP64
additions of the grid cells.  Corrections, padding, the centred FFTs and
the crop are the serial code of ``gridding`` on the whole grid.

Workers are forked, so the inputs (set as module globals before the pool
starts) are shared with them without copies.
"""

import multiprocessing as mp
import os

import numpy as np

from . import decentral, gridding
from .es_kernel import correction, es_beta
from .geometry import grid_coord

_G = {}  # inputs of the current parallel step, inherited by the forked workers
MIN_CHUNK = 65536  # visibilities per chunk at least


def default_workers():
    """The cores this process may use, capped by OMP_NUM_THREADS when that
    is set (a machine's share of its cores for one job)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    cap = os.environ.get("OMP_NUM_THREADS", "")
    if cap.isdigit() and int(cap) > 0:
        n = min(n, int(cap))
    return max(1, n)


def _chunks(m, workers):
    k = max(1, min(workers, (m + MIN_CHUNK - 1) // MIN_CHUNK))
    edges = np.linspace(0, m, k + 1).astype(np.int64)
    return [(int(a), int(b)) for a, b in zip(edges[:-1], edges[1:]) if b > a]


def _degrid_chunk(ab):
    a, b = ab
    return gridding.degrid(_G["grid"], _G["gx"][a:b], _G["gy"][a:b], _G["W"], _G["beta"])


def _grid_chunk(ab):
    a, b = ab
    return gridding.grid_vis(_G["vis"][a:b], _G["gx"][a:b], _G["gy"][a:b], _G["ng"], _G["W"],
                             _G["beta"])


def _map(fn, jobs, workers):
    if workers <= 1 or len(jobs) == 1:
        return [fn(j) for j in jobs]
    ctx = mp.get_context("fork")
    with ctx.Pool(min(workers, len(jobs))) as pool:
        return list(pool.imap(fn, jobs))  # chunk order


def forward(image, gx, gy, n_grid, support, beta, workers):
    """gridding.forward with the degridding split over chunks."""
    n = image.shape[0]
    psi = correction(n, n_grid, support, beta)
    corrected = np.asarray(image, dtype=np.complex128) / np.outer(psi, psi)
    _G.update(grid=gridding.centred_fft2(gridding.pad_centre(corrected, n_grid)), gx=gx, gy=gy,
              W=support, beta=beta)
    try:
        parts = _map(_degrid_chunk, _chunks(len(gx), workers), workers)
    finally:
        _G.clear()
    return np.concatenate(parts)


def grid_vis(vis, gx, gy, n_grid, support, beta, workers):
    """gridding.grid_vis with the visibilities split over chunks; the chunk
    grids are added in chunk order."""
    _G.update(vis=np.asarray(vis, np.complex128), gx=gx, gy=gy, ng=n_grid, W=support, beta=beta)
    try:
        jobs = _chunks(len(gx), workers)
        if workers <= 1 or len(jobs) == 1:
            parts = [_grid_chunk(j) for j in jobs]
            out = parts[0]
            for p in parts[1:]:
                out = out + p
            return out
        ctx = mp.get_context("fork")
        out = None
        with ctx.Pool(min(workers, len(jobs))) as pool:
            for p in pool.imap(_grid_chunk, jobs):
                out = p if out is None else out + p
        return out
    finally:
        _G.clear()


def adjoint(vis, gx, gy, n_img, n_grid, support, beta, workers):
    """gridding.adjoint with the gridding split over chunks."""
    psi = correction(n_img, n_grid, support, beta)
    g = grid_vis(vis, gx, gy, n_grid, support, beta, workers)
    return gridding.crop_centre(gridding.centred_ifft2(g), n_img) / np.outer(psi, psi)


def residual_image(u, v, vis, w, model, cell, support=8, workers=None, sigma=2):
    """imaging.residual_image (Eq. 2) over worker processes."""
    workers = default_workers() if workers is None else workers
    n = model.shape[0]
    ng = int(round(sigma * n))
    beta = es_beta(support)
    gx, gy = grid_coord(u, ng, cell), grid_coord(v, ng, cell)
    pred = (forward(model, gx, gy, ng, support, beta, workers) if np.any(model)
            else np.zeros(len(u), np.complex128))
    r = np.asarray(vis, np.complex128) - pred
    img = adjoint(np.asarray(w, np.float64) * r, gx, gy, n, ng, support, beta, workers).real
    return img / np.sum(w), pred


def psf2(u, v, w, n_img, cell, support=8, workers=None, sigma=2):
    """imaging.psf2 (2N x 2N, peak 1 at (N, N)) over worker processes."""
    workers = default_workers() if workers is None else workers
    n2 = 2 * n_img
    ng = int(round(sigma * n2))
    beta = es_beta(support)
    gx, gy = grid_coord(u, ng, cell), grid_coord(v, ng, cell)
    img = adjoint(np.asarray(w, np.float64), gx, gy, n2, ng, support, beta, workers).real
    return img / np.sum(w)


def decentral_cycle(u, v, vis, w, masks, model, rho, psfs, gammas, mus, ell, delta, cell,
                    support=8, workers=None):
    """One decentralized major cycle of both nodes (Eq. 2, then Eq. 7):
    per node k, i~_k = residual of model[k] on its visibilities and D_k =
    gamma_k Gamma_own i~_k + mu_k H_other rho[k].  Returns (D, i~) lists."""
    outs, locs = [], []
    for k, own in enumerate(("L", "H")):
        m = masks[k]
        loc, _ = residual_image(u[m], v[m], vis[m], w[m], model[k], cell, support, workers)
        locs.append(loc)
        outs.append(decentral.compose_dirty(loc, rho[k], psfs[1 - k], ell, delta, own,
                                            gammas[k], mus[k]))
    return outs, locs


__all__ = ["default_workers", "forward", "grid_vis", "adjoint", "residual_image", "psf2",
           "decentral_cycle"]
