"""Seeded synthetic workloads shaped like the paper's data sets.

The paper's data (Table 1: Sgr B2, Sgr C, HL Tau, Cygnus A) are not
available, so every input is synthesised here from a seed.  This module
holds no step of the imaging method: it lays out an array, runs textbook
Earth-rotation synthesis to get (u, v, w), places point and Gaussian
sources, and evaluates each source's analytic Fourier transform plus
complex Gaussian noise.  Both the HIP library (through the tests and the
benchmark) and the CPU oracle consume exactly the arrays it returns.

Recipe:
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


def make(name="tiny", seed=None, n_time=None, with_noise=True, sky_scale=1.0, device=None):
    """Generate a workload.  Returns a dict with

    uvw [M, 3] float64 metres, vis [M] complex128 (complex64 for the c64
    workloads), weight [M] float32 (ones), freq_hz, cell (rad), n_img,
    truth [N, N] float64 (Jy/pixel), sources.

    With ``device`` (a torch device) the source sums of each time step are
    evaluated there in FP64 (batches of time steps), for the large
    workloads; the arrays returned are numpy arrays either way and the
    two evaluations differ only in FP64 rounding.
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
    if device is not None:
        _vis_device(vis, auvw / lam, bi, bj, l0, m0, flux, sig * cell, wl.n_points, device)
    for t in range(n_time if device is None else 0):
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


def _vis_device(out, auv, bi, bj, l0, m0, flux, sig_rad, n_points, device, batch=16):
    """The per-time source sums of ``make`` with torch on ``device`` (FP64):
    points through the antenna phasors, Gaussians with their envelopes."""
    import torch
    n_time, n_ant = auv.shape[0], auv.shape[1]
    n_bl = len(bi)
    t_l0 = torch.tensor(l0, dtype=torch.float64, device=device)
    t_m0 = torch.tensor(m0, dtype=torch.float64, device=device)
    t_flux = torch.tensor(flux, dtype=torch.float64, device=device)
    t_sig = torch.tensor(sig_rad, dtype=torch.float64, device=device)
    t_bi = torch.tensor(bi, device=device)
    t_bj = torch.tensor(bj, device=device)
    pts, gss = slice(0, n_points), slice(n_points, len(flux))
    for t0 in range(0, n_time, batch):
        t1 = min(n_time, t0 + batch)
        a = torch.tensor(auv[t0:t1], dtype=torch.float64, device=device)   # [T, A, 3]
        phase = -2.0 * np.pi * (a[:, :, 0:1] * t_l0 + a[:, :, 1:2] * t_m0)  # [T, A, S]
        ph = torch.polar(torch.ones_like(phase), phase)                     # complex128
        left = (ph[:, :, pts] * t_flux[pts]).contiguous()
        right = ph[:, :, pts].conj().transpose(1, 2).contiguous()           # [T, S, A]
        vt = torch.bmm(left, right)[:, t_bj, t_bi]                          # [T, B]
        if len(flux) > n_points:
            ub = a[:, t_bj, 0] - a[:, t_bi, 0]
            vb = a[:, t_bj, 1] - a[:, t_bi, 1]
            q = ub * ub + vb * vb                                           # [T, B]
            env = torch.exp(-2.0 * np.pi ** 2 * q[:, :, None] * (t_sig[gss] ** 2))  # [T, B, G]
            pg = ph[:, t_bj, gss] * ph[:, t_bi, gss].conj()
            vt = vt + ((env * pg) * t_flux[gss]).sum(dim=2)
        out[t0 * n_bl:t1 * n_bl] = vt.reshape(-1).cpu().numpy()
        del a, phase, ph, left, right, vt


def random_uv_cells(m, n_grid, rng, frac=1.0 / 3.0):
    """Uniform random grid-relative coordinates |u|,|v| <= frac * Ng cells
    (for unit tests of the operator); returned in cells from the centre."""
    return rng.uniform(-frac * n_grid, frac * n_grid, (2, m))


# Frequency channels of the 256-antenna array: 0.95 - 1.75 GHz, each flagged
# uniformly at random with its own fraction in [0, 0.6], image sizes drawn
# from 512 / 1024 / 2048 (the batched-channel workload).
CHANNELS = dict(n_chan=64, n_ant=256, radius_m=4000.0, n_time=480, f_lo=0.95e9, f_hi=1.75e9,
                flag_max=0.6, sizes=(512, 1024, 2048), n_points=200, seed=5, t_min=240)


def make_channels(n_chan=64, n_ant=256, radius_m=4000.0, n_time=480, f_lo=0.95e9, f_hi=1.75e9,
                  flag_max=0.6, sizes=(512, 1024, 2048), n_points=200, seed=5, device=None,
                  t_min=None):
    """Multi-channel workload over one array and one time range.

    Returns dict(uvw [M, 3] float64 metres shared by all channels, channels =
    list of dict(freq_hz, cell, n_img, flag uint8 [M], vis complex64 [M],
    flag_frac, n_time)).  Channel c is at f_lo + (f_hi - f_lo) c / (n_chan - 1); its
    cell is 1 / (3 max |u|) at that frequency.  With ``t_min`` each channel
    keeps its own number of time samples T_c, uniform in {t_min .. n_time}:
    its samples past the first T_c time steps are flagged (an uneven
    observation length per channel).  The sky is n_points point
    sources with log-uniform fluxes in [1 mJy, 1 Jy] and spectral index -0.7
    (reference 1.4 GHz), placed in the central 80 % of the smallest field of
    view of the band; noise sigma 1 mJy.  With ``device`` (a torch cuda
    device) uvw, flag and vis are torch tensors evaluated on that device,
    else numpy arrays (small cases: the per-time antenna phasors are formed
    on the CPU)."""
    rng = np.random.default_rng(seed)
    xyz = antenna_xyz(n_ant, radius_m, rng)
    ha = hour_angles(n_time)
    auvw = antenna_uvw(xyz, ha)                       # [T, A, 3]
    bi, bj = baselines(n_ant)
    uvw = (auvw[:, bj, :] - auvw[:, bi, :]).reshape(-1, 3)
    m_vis = uvw.shape[0]
    freqs = f_lo + (f_hi - f_lo) * np.arange(n_chan) / max(n_chan - 1, 1)
    umax_m = max(np.abs(uvw[:, 0]).max(), np.abs(uvw[:, 1]).max())
    cells = 1.0 / (3.0 * umax_m * freqs / C_LIGHT)
    n_img = [int(sizes[k]) for k in rng.integers(0, len(sizes), n_chan)]
    flag_frac = rng.uniform(0.0, flag_max, n_chan)
    # sky in direction cosines inside the smallest field of view
    fov = min(sizes) * cells.min()
    l0 = rng.uniform(-0.4, 0.4, n_points) * fov
    m0 = rng.uniform(-0.4, 0.4, n_points) * fov
    flux0 = 10.0 ** rng.uniform(-3.0, 0.0, n_points)
    seeds = rng.integers(0, 2 ** 31 - 1, n_chan)
    t_keep = (rng.integers(t_min, n_time + 1, n_chan) if t_min is not None
              else np.full(n_chan, n_time))
    chans = []
    if device is not None:
        import torch
        t_auvw = torch.tensor(auvw, dtype=torch.float64, device=device)
        t_l0 = torch.tensor(l0, device=device)
        t_m0 = torch.tensor(m0, device=device)
        t_bi = torch.tensor(bi, device=device)
        t_bj = torch.tensor(bj, device=device)
        uvw_out = torch.tensor(uvw, dtype=torch.float64, device=device)
    for c in range(n_chan):
        f = freqs[c]
        lam = C_LIGHT / f
        flux = flux0 * (f / 1.4e9) ** -0.7
        crng = np.random.default_rng(int(seeds[c]))
        if device is None:
            vis = np.empty(m_vis, np.complex128)
            n_bl = len(bi)
            for t in range(n_time):
                ph = np.exp(-2j * np.pi * (np.outer(auvw[t, :, 0] / lam, l0)
                                           + np.outer(auvw[t, :, 1] / lam, m0)))
                vmat = (ph * flux) @ ph.conj().T
                vis[t * n_bl:(t + 1) * n_bl] = vmat[bj, bi]
            vis += 1e-3 * (crng.standard_normal(m_vis) + 1j * crng.standard_normal(m_vis))
            flag = (crng.random(m_vis) < flag_frac[c]).astype(np.uint8)
            flag[int(t_keep[c]) * len(bi):] = 1
            vis = vis.astype(np.complex64)
        else:
            import torch
            phase = -2.0 * np.pi * (t_auvw[:, :, 0:1] / lam * t_l0 + t_auvw[:, :, 1:2] / lam * t_m0)
            ph = torch.polar(torch.ones_like(phase), phase).to(torch.complex64)   # [T, A, S]
            t_flux = torch.tensor(flux, dtype=torch.float32, device=device)
            right = ph.conj().transpose(1, 2).contiguous()                         # [T, S, A]
            vmat = torch.bmm(ph * t_flux, right)                                  # [T, A, A]
            vis = vmat[:, t_bj, t_bi].reshape(-1)
            g = torch.Generator(device=device)
            g.manual_seed(int(seeds[c]))
            noise = torch.randn(2, m_vis, generator=g, device=device, dtype=torch.float32)
            vis = vis + 1e-3 * torch.complex(noise[0], noise[1])
            flag = (torch.rand(m_vis, generator=g, device=device) < flag_frac[c]).to(torch.uint8)
            flag[int(t_keep[c]) * len(bi):] = 1
            del phase, ph, right, vmat, noise
        chans.append(dict(freq_hz=float(f), cell=float(cells[c]), n_img=n_img[c], flag=flag,
                          vis=vis, flag_frac=float(flag_frac[c]), n_time=int(t_keep[c])))
    return dict(uvw=uvw if device is None else uvw_out, channels=chans, n_vis=m_vis,
                n_ant=n_ant, n_time=n_time)


def make_requests(n_req, seed=6, n_ant=256, radius_m=4000.0, vis_range=(1.0e6, 5.0e7),
                  sizes=(512, 1024, 2048), freq_hz=1.4e9, n_points=100, n_gauss=10,
                  gauss_sigma_px=(2.0, 8.0), device="cuda"):
    """Imaging requests of mixed shape for the serving workload.

    Request r observes with the n_ant-antenna array for T_r time samples
    over [-2 h, +2 h] (its own hour-angle grid), T_r = M_r / n_baselines
    rounded, with M_r log-uniform in ``vis_range``; its image side is drawn
    from ``sizes`` and its cell is 1 / (3 max |u|) of its own samples.  Its
    sky has n_points points and n_gauss circular Gaussians (sigma in pixels
    uniform in gauss_sigma_px), pixel-centred in the central 80 % of its
    image, fluxes log-uniform in [1 mJy, 1 Jy]; noise sigma 1 mJy.  The
    source sums are evaluated with torch on ``device`` in complex64.
    Returns a list of dict(uvw [M_r, 3] float64, vis [M_r] complex64 (both
    device tensors), freq_hz, cell, n_img, n_time, n_vis)."""
    import torch
    rng = np.random.default_rng(seed)
    xyz = antenna_xyz(n_ant, radius_m, rng)
    bi, bj = baselines(n_ant)
    t_bi = torch.tensor(bi, device=device)
    t_bj = torch.tensor(bj, device=device)
    n_bl = len(bi)
    lam = C_LIGHT / freq_hz
    out = []
    for _ in range(n_req):
        m_r = float(np.exp(rng.uniform(np.log(vis_range[0]), np.log(vis_range[1]))))
        n_time = max(1, int(round(m_r / n_bl)))
        n = int(sizes[rng.integers(0, len(sizes))])
        auvw = antenna_uvw(xyz, hour_angles(n_time))                  # [T, A, 3] metres
        t_auvw = torch.tensor(auvw, dtype=torch.float64, device=device)
        uvw = (t_auvw[:, t_bj, :] - t_auvw[:, t_bi, :]).reshape(-1, 3)
        umax = float(torch.max(torch.abs(uvw[:, :2])).item()) / lam
        cell = 1.0 / (3.0 * umax)
        lo, hi = int(0.1 * n), int(0.9 * n)
        n_src = n_points + n_gauss
        ix = rng.integers(lo, hi, n_src)
        iy = rng.integers(lo, hi, n_src)
        flux = 10.0 ** rng.uniform(-3.0, 0.0, n_src)
        sig = rng.uniform(gauss_sigma_px[0], gauss_sigma_px[1], n_gauss) * cell
        l0 = torch.tensor((ix - n // 2) * cell, device=device)
        m0 = torch.tensor((iy - n // 2) * cell, device=device)
        t_flux = torch.tensor(flux, dtype=torch.float32, device=device)
        t_sig = torch.tensor(sig, device=device)
        vis = torch.empty(n_time * n_bl, dtype=torch.complex64, device=device)
        pts, gss = slice(0, n_points), slice(n_points, n_src)
        for t0 in range(0, n_time, 32):
            t1 = min(n_time, t0 + 32)
            a = t_auvw[t0:t1] / lam                                         # [T, A, 3]
            phase = -2.0 * np.pi * (a[:, :, 0:1] * l0 + a[:, :, 1:2] * m0)  # [T, A, S]
            ph = torch.polar(torch.ones_like(phase), phase).to(torch.complex64)
            left = (ph[:, :, pts] * t_flux[pts]).contiguous()
            right = ph[:, :, pts].conj().transpose(1, 2).contiguous()
            vt = torch.bmm(left, right)[:, t_bj, t_bi]
            ub = a[:, t_bj, 0] - a[:, t_bi, 0]
            vb = a[:, t_bj, 1] - a[:, t_bi, 1]
            q = (ub * ub + vb * vb)
            env = torch.exp(-2.0 * np.pi ** 2 * q[:, :, None] * (t_sig ** 2)).to(torch.float32)
            pg = ph[:, t_bj, gss] * ph[:, t_bi, gss].conj()
            vt = vt + ((env * pg) * t_flux[gss]).sum(dim=2)
            vis[t0 * n_bl:t1 * n_bl] = vt.reshape(-1)
            del a, phase, ph, left, right, vt, ub, vb, q, env, pg
        g = torch.Generator(device=device)
        g.manual_seed(int(rng.integers(0, 2 ** 31 - 1)))
        noise = torch.randn(2, vis.shape[0], generator=g, device=device, dtype=torch.float32)
        vis += 1e-3 * torch.complex(noise[0], noise[1])
        del noise, t_auvw
        out.append(dict(uvw=uvw, vis=vis, freq_hz=freq_hz, cell=cell, n_img=n, n_time=n_time,
                        n_vis=int(vis.shape[0])))
    return out
