"""Shared pieces of the GPU tests: seeded inputs and the oracle's answers."""

import functools
import sys

import numpy as np

from oracle import decentral, geometry, imaging
from paper_2507_22128_amd import synth


def rel(a, b):
    a = np.asarray(a, np.complex128).ravel()
    b = np.asarray(b, np.complex128).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=8)
def workload(name, n_time=None, seed=None):
    return synth.make(name, n_time=n_time, seed=seed)


def uv(d):
    return geometry.uv_lambda(d["uvw"], d["freq_hz"])


def random_model(n, rng, n_points=30, smooth=True):
    """A model image with point components and a smooth blob (f64)."""
    m = np.zeros((n, n))
    ix = rng.integers(n // 8, n - n // 8, n_points)
    iy = rng.integers(n // 8, n - n // 8, n_points)
    np.add.at(m, (iy, ix), rng.uniform(0.05, 0.5, n_points))
    if smooth:
        yy, xx = np.mgrid[0:n, 0:n]
        m += 0.2 * np.exp(-((xx - 0.6 * n) ** 2 + (yy - 0.4 * n) ** 2) / (2 * (0.03 * n) ** 2))
    return m


def oracle_weights(d, n, valid=None, uniform=True):
    u, v = uv(d)
    if uniform:
        return imaging.uniform_weights(u, v, n, d["cell"], valid=valid)
    w = np.ones(len(u))
    if valid is not None:
        w[~valid] = 0
    return w


@functools.lru_cache(maxsize=4)
def oracle_inputs(name, n_time=None, partitions=1, model_scale=0.0):
    """Inputs for teacher-forced minor cycles, all from the oracle (FP64):
    per partition (one: the whole set; two: the median split of the
    oracle's partition) the residual image of model_scale * truth (Eq. 2)
    and the 2N x 2N PSF; with the split's ell and the partitions' weight
    sums."""
    d = workload(name, n_time=n_time)
    n = d["n_img"]
    u, v = uv(d)
    w = oracle_weights(d, n)
    if partitions == 1:
        masks, ell = [np.ones(len(u), bool)], None
    else:
        low, high, ell = imaging.partition(u, v, n, d["cell"])
        masks = [low, high]
    model = model_scale * d["truth"]
    out = {"ell": ell, "sum_w": [float(w[m].sum()) for m in masks], "resid": [], "psf": []}
    for m in masks:
        r, _ = imaging.residual_image(u[m], v[m], d["vis"][m], w[m], model, d["cell"])
        out["resid"].append(r)
        out["psf"].append(imaging.psf2(u[m], v[m], w[m], n, d["cell"]))
    return out


def ibar_from_components(comps, scales, n):
    """The minor cycle's model ibar rebuilt from its components (scale index,
    iy, ix, amplitude), placed in order as the oracle's minor cycle places
    them (bit for bit the same FP64 sums)."""
    from oracle import msclean
    kern = [msclean.scale_kernel(s) for s in scales]
    ibar = np.zeros((n, n))
    for s, iy, ix, a in comps:
        msclean.add_component(ibar, kern[int(s)], int(iy), int(ix), float(a))
    return ibar


def f32(a):
    """Round to float32 (the precision both sides of a teacher-forced test
    receive), kept as float64 for the oracle."""
    return np.asarray(a, np.float32).astype(np.float64)


def to_dev(x, dtype="float32"):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=getattr(torch, dtype), device="cuda")


def to_np(t):
    return t.detach().cpu().numpy()


__all__ = ["rel", "say", "workload", "uv", "random_model", "oracle_weights", "oracle_inputs",
           "ibar_from_components", "f32", "to_dev", "to_np", "decentral", "imaging", "geometry"]
