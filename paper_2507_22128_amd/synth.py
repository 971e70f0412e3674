"""Seeded synthetic workloads shaped like the paper's data sets.

The paper's data (Table 1: Sgr B2, Sgr C, HL Tau, Cygnus A) are not
available, so every input is synthesised here from a seed.  This module
holds no step of the imaging method: it lays out an array, runs textbook
Earth-rotation synthesis to get (u, v, w), places point and Gaussian
sources, and evaluates each source's analytic Fourier transform plus
complex Gaussian noise.  Both the HIP library (through the tests and the
benchmark) and the CPU oracle consume exactly the arrays it returns.

Recipe (also in the design doc):
* antennas uniform over a disk (radius R sqrt(U), angle 2 pi U'), flat,
  at latitude -30.7 deg; all i < j baselines;
* phase centre at declination -30 deg, hour angles at the midpoints of
  n_time equal steps over [-2 h, +2 h]; visibilities in time-major order;
* pixel size 1 / (3 max(|u|, |v|)) so the sampled uv disk fills two thirds
  of a 2x padded grid's half-width;
* point sources at pixel centres uniform in the central 80 % of the image,
  Gaussians (circular, sigma in pixels) likewise, fluxes log-uniform in
  [1 mJy, 1 Jy]; noise sigma 1 mJy per real and imaginary part;
* w is produced and ignored by the coplanar imager.
"""

import dataclasses

import numpy as np

C_LIGHT = 299792458.0


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n_ant: int
    radius_m: float
    n_time: int
    freq_hz: float
    n_img: int
    n_points: int
    n_gauss: int
    gauss_sigma_px: tuple
    seed: int
    vis_dtype: str          # "c128" or "c64"
    partitions: int


WORKLOADS = {
    # 64 antennas in a 2 km disk, 2016 baselines x 60 times, 256^2 image.
    "tiny": Workload("tiny", 64, 1000.0, 60, 1.4e9, 256, 20, 3, (2.0, 8.0), 1, "c128", 1),
    # 256 antennas in an 8 km disk, 32640 baselines x 480 times, 1024^2 image,
    # two partitions split at the median |uv|.
    "decentral": Workload("decentral", 256, 4000.0, 480, 1.4e9, 1024, 200, 30, (2.0, 8.0), 2, "c64", 2),
    # same array, 2048^2 image, 32640 x 1532 = 50,004,480 visibilities.
    "convex": Workload("convex", 256, 4000.0, 1532, 1.4e9, 2048, 500, 50, (4.0, 40.0), 3, "c64", 2),
}


def antenna_xyz(n_ant, radius_m, rng, lat_deg=-30.7):
    """Antenna positions (X, Y, Z) in metres for a flat disk array."""
    r = radius_m * np.sqrt(rng.random(n_ant))
    th = 2.0 * np.pi * rng.random(n_ant)
    east, north, up = r * np.cos(th), r * np.sin(th), np.zeros(n_ant)
    lat = np.deg2rad(lat_deg)
    x = -np.sin(lat) * north + np.cos(lat) * up
    y = east
    z = np.cos(lat) * north + np.sin(lat) * up
    return np.stack([x, y, z], axis=1)


def hour_angles(n_time, span_h=4.0):
    step = span_h / n_time
    h = -span_h / 2.0 + (np.arange(n_time) + 0.5) * step
    return np.deg2rad(15.0 * h)


def antenna_uvw(xyz, ha, dec_deg=-30.0):
    """Per-antenna (u, v, w) in metres, shape [n_time, n_ant, 3]."""
    dec = np.deg2rad(dec_deg)
    sh, ch = np.sin(ha)[:, None], np.cos(ha)[:, None]
    x, y, z = xyz[:, 0][None], xyz[:, 1][None], xyz[:, 2][None]
    u = sh * x + ch * y
    v = -np.sin(dec) * ch * x + np.sin(dec) * sh * y + np.cos(dec) * z
    w = np.cos(dec) * ch * x - np.cos(dec) * sh * y + np.sin(dec) * z
    return np.stack([u, v, w], axis=2)


def baselines(n_ant):
    i, j = np.triu_indices(n_ant, k=1)
    return i.astype(np.int64), j.astype(np.int64)


def make(name="tiny", seed=None, n_time=None, with_noise=True, sky_scale=1.0):
    """Generate a workload.  Returns a dict with

    uvw [M, 3] float64 metres, vis [M] complex128, weight [M] float32 (ones),
    freq_hz, cell (rad), n_img, truth [N, N] float64 (Jy/pixel), sources.
    """
    wl = WORKLOADS[name]
    rng = np.random.default_rng(wl.seed if seed is None else seed)
    n_time = wl.n_time if n_time is None else n_time
    xyz = antenna_xyz(wl.n_ant, wl.radius_m, rng)
    ha = hour_angles(n_time)
    auvw = antenna_uvw(xyz, ha)                       # [T, A, 3] metres
    bi, bj = baselines(wl.n_ant)
    uvw = (auvw[:, bj, :] - auvw[:, bi, :]).reshape(-1, 3)
    lam = C_LIGHT / wl.freq_hz
    umax = max(np.abs(uvw[:, 0]).max(), np.abs(uvw[:, 1]).max()) / lam
    cell = 1.0 / (3.0 * umax)
    n = wl.n_img

    # sky: pixel-centred components in the central 80 % box
    lo, hi = int(0.1 * n), int(0.9 * n)
    n_src = wl.n_points + wl.n_gauss
    ix = rng.integers(lo, hi, n_src)
    iy = rng.integers(lo, hi, n_src)
    flux = sky_scale * 10.0 ** rng.uniform(-3.0, 0.0, n_src)
    sig = np.zeros(n_src)
    sig[wl.n_points:] = rng.uniform(wl.gauss_sigma_px[0], wl.gauss_sigma_px[1], wl.n_gauss)
    l0 = (ix - n // 2) * cell
    m0 = (iy - n // 2) * cell

    # visibilities: per time step, point sources through the antenna phasors
    # (V_ij = sum_s S_s P_js conj(P_is)), Gaussians with their envelope.
    n_bl = len(bi)
    vis = np.empty(n_time * n_bl, np.complex128)
    pts = slice(0, wl.n_points)
    gss = slice(wl.n_points, n_src)
    for t in range(n_time):
        ua = auvw[t, :, 0] / lam
        va = auvw[t, :, 1] / lam
        ph = np.exp(-2j * np.pi * (np.outer(ua, l0) + np.outer(va, m0)))  # [A, S]
        vmat = (ph[:, pts] * flux[pts]) @ ph[:, pts].conj().T            # [A, A]
        vt = vmat[bj, bi]
        if wl.n_gauss:
            ub = ua[bj] - ua[bi]
            vb = va[bj] - va[bi]
            q = ub * ub + vb * vb
            sg = sig[gss] * cell
            env = np.exp(-2.0 * np.pi ** 2 * np.outer(q, sg * sg))        # [B, G]
            phg = ph[:, gss]
            pg = phg[bj] * phg[bi].conj()
            vt = vt + (env * pg) @ flux[gss]
        vis[t * n_bl:(t + 1) * n_bl] = vt
    if with_noise:
        vis += 1e-3 * (rng.standard_normal(vis.size) + 1j * rng.standard_normal(vis.size))

    truth = np.zeros((n, n))
    np.add.at(truth, (iy[pts], ix[pts]), flux[pts])
    yy, xx = np.mgrid[0:n, 0:n]
    for s in range(wl.n_points, n_src):
        g = np.exp(-((xx - ix[s]) ** 2 + (yy - iy[s]) ** 2) / (2.0 * sig[s] ** 2))
        truth += flux[s] * g / (2.0 * np.pi * sig[s] ** 2)
    if wl.vis_dtype == "c64":
        vis = vis.astype(np.complex64)
    return dict(name=name, uvw=uvw, vis=vis, weight=np.ones(len(vis), np.float32),
                freq_hz=wl.freq_hz, cell=cell, n_img=n, truth=truth,
                sources=dict(ix=ix, iy=iy, flux=flux, sigma_px=sig), workload=wl)


def random_uv_cells(m, n_grid, rng, frac=1.0 / 3.0):
    """Uniform random grid-relative coordinates |u|,|v| <= frac * Ng cells
    (for unit tests of the operator); returned in cells from the centre."""
    return rng.uniform(-frac * n_grid, frac * n_grid, (2, m))
