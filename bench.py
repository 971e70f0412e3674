#!/usr/bin/env python3
"""Benchmark of the major-cycle measurement operator on one MI355X.

A step is one decentralized major cycle of a two-partition workload: for
each node (V_L and V_H, concurrently) the model is transformed to the
grid, every visibility is degridded, its weighted residual gridded, the
grid flushed and transformed back to the residual image (Eq. 2), and the
residual is composed with the other node's aggregate through the other
node's PSF (Eq. 7).  Preparation (weighting, partition, sort) and the PSFs
are one-time work of imager_create and are timed separately (create_ms).

The headline workload is the largest single-GPU one (50,004,480
visibilities, 2048^2 image); the 15.7M-visibility 1024^2 workload is
measured the same way as an extra.  Every timed configuration's outputs are
compared with the FP64 oracle run over the same full partitions, which is
also timed on the host's cores as the CPU baseline.

Prints one JSON line.  ``value`` is whole-job throughput: unflagged
visibilities of the data set per second of major cycle (Mvis/s), inputs
resident in HBM.
"""

import argparse
import json
import os
import sys
import time

METRIC = "major-cycle Mvis/s (grid+degrid) at ≤1e-5 rel err, %HBM roofline; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
# MI355X published dense FP32 matrix peak (TFLOP/s).  The de/gridding
# products run as FP32 MFMA; on gfx950 these issue through the same pipe as
# vector FP32, so 157.3 is the ceiling of the whole kernel's arithmetic.
FP32_PEAK_MATRIX = 157.3


# HBM bytes per launch of the fused de/grid kernel, per workload, from the
# FETCH_SIZE / WRITE_SIZE counter runs with the copy-kernel calibration
# (profiles/convex_hbm_traffic.md), valid only for the kernel source the
# counters were taken on.
KWINDOW_TRAFFIC = {
    "convex": {"src": "paper_2507_22128_amd/csrc/degrid_grid.hip",
               "sha256_16": "a8236ee97984adf6",
               "bytes_per_launch": (340044.3 * 1024 * 2.0 + 101240.0 * 1024 * 1.0)},
}


def measured_traffic(name):
    import hashlib
    t = KWINDOW_TRAFFIC.get(name)
    if t is None:
        return None
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), t["src"])
    with open(path, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    return t["bytes_per_launch"] if sha == t["sha256_16"] else None


def log(msg):
    sys.stderr.write("[bench] %s\n" % msg)
    sys.stderr.flush()


def flops_per_vis(w):
    """Arithmetic of one visibility in the fused de/grid kernel (W taps/axis):
    2W kernel weights (6 flop each incl. sqrt and exp), degrid 4W^2 + 4W,
    residual 4, gridding 2W + 2W^2 products and 2W^2 accumulations."""
    return 8 * w * w + 18 * w + 4


def oracle_cycle(d, outs, locs, workers):
    """The FP64 oracle, as it stands, on the full timed partitions: weights,
    partition and both PSFs (one-time work, untimed, as the library's
    create), then one decentralized major cycle of both nodes (Eq. 2 for
    each node's visibilities, then Eq. 7) with the same model and aggregate
    images as the timed steps, timed.  Gridding and degridding run over
    visibility chunks on ``workers`` host processes (oracle.pool); the FFTs
    are NumPy's.  Returns the cpu_baseline object and the errors of the
    timed GPU outputs against the oracle's."""
    import numpy as np
    from oracle import decentral, geometry, imaging, pool
    n = d["n_img"]
    cell = d["cell"]
    t0 = time.perf_counter()
    u, v = geometry.uv_lambda(d["uvw"], d["freq_hz"])
    w = imaging.uniform_weights(u, v, n, cell)
    low, high, ell = imaging.partition(u, v, n, cell)
    masks = (low, high)
    psfs = [pool.psf2(u[m], v[m], w[m], n, cell, workers=workers) for m in masks]
    t_setup = time.perf_counter() - t0
    wsum = [w[m].sum() for m in masks]
    gm = [decentral.weights_schedule(2, wsum[p], wsum[1 - p]) for p in (0, 1)]
    model = [0.5 * d["truth"]] * 2
    rho = [0.01 * d["truth"]] * 2
    t0 = time.perf_counter()
    ref_outs, ref_locs = pool.decentral_cycle(u, v, d["vis"], w, masks, model, rho, psfs,
                                              [g[0] for g in gm], [g[1] for g in gm], ell, 1.0,
                                              cell, workers=workers)
    t_cpu = time.perf_counter() - t0
    relerr = lambda a, b: float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))
    err = {"composed_rel_l2": [relerr(outs[p], ref_outs[p]) for p in (0, 1)],
           "local_rel_l2": [relerr(locs[p], ref_locs[p]) for p in (0, 1)]}
    err["max_rel_l2"] = max(err["composed_rel_l2"] + err["local_rel_l2"])
    err["tolerance"] = 1e-5
    err["pass"] = bool(err["max_rel_l2"] <= 1e-5)
    try:
        cpu_model = [ln.split(":", 1)[1].strip() for ln in open("/proc/cpuinfo")
                     if ln.startswith("model name")][0]
    except (OSError, IndexError):
        cpu_model = "unknown"
    base = {
        "value": round(len(u) / t_cpu / 1e6, 4),
        "unit": "Mvis/s",
        "cores": int(workers),
        "kind": "oracle",
        "sample": "the whole timed workload: one decentralized major cycle of both partitions "
                  "(%d visibilities; Eq. 2 per node, then Eq. 7) with the timed step's model "
                  "and aggregate images, FP64 NumPy/SciPy oracle, de/gridding over visibility "
                  "chunks on %d processes, NumPy FFTs; %.1f s (weights, partition and PSFs, "
                  "one-time like the library's create, %.1f s more, untimed)"
                  % (len(u), workers, t_cpu, t_setup),
        "cpu_model": cpu_model,
        "seconds": round(t_cpu, 2),
    }
    return base, err


def minor_cycles(h, info, model, rho, gammas, mus, n, msclean=True):
    """Device time of the minor cycles on node V_L's cycle-2 problem of the
    workload: multi-scale CLEAN (S = {0, 4, 12} px, gain 0.1, K = 2000,
    FP64) on the composed dirty image and PSF of Eq. 7 (with ``msclean``),
    and FISTA (db8, 3 levels, 200 iterations, 30 power iterations, lambda =
    1e-3 max |i~|, FP64 transforms) on the node's residual and aggregate
    (Eq. 5), plus FISTA over the 8-basis dictionary (50 iterations)."""
    import numpy as np
    import torch
    out = {}
    if not msclean:
        return _fista_cycles(h, model, rho, gammas, mus, n, out)
    dirty = h.major_cycle(0, model[0], rho[0], gammas[0], mus[0])
    psf = h.composed_psf(0, gammas[0], mus[0])
    h.minor_cycle_msclean(0, dirty, psf, [0, 4, 12], niter=10)  # work area, warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, comps, _ = h.minor_cycle_msclean(0, dirty, psf, [0, 4, 12], gain=0.1, niter=2000)
    t_msc = time.perf_counter() - t0
    n_int = 3  # smoothed residuals kept (scale 0 is in S)
    bytes_iter = 24.0 * n_int * n * n  # read R_t, read B_{s*t}, write R_t (FP64) per iteration
    out["msclean"] = {
        "ms": round(1e3 * t_msc, 2), "iterations": int(len(comps)),
        "us_per_iteration": round(1e6 * t_msc / max(len(comps), 1), 2),
        "update_gbs": round(bytes_iter * len(comps) / t_msc / 1e9, 1),
        "update_hbm_frac": round(bytes_iter * len(comps) / t_msc / 1e9 / HBM_PEAK_GBS, 4),
        "config": "node V_L, cycle-2 composed dirty / PSF (Eq. 7), %d^2, S = {0, 4, 12} px, "
                  "gain 0.1, K = 2000, FP64" % n}
    return _fista_cycles(h, model, rho, gammas, mus, n, out)


def _fista_cycles(h, model, rho, gammas, mus, n, out):
    import numpy as np
    import torch
    local = torch.empty((n, n), device="cuda")
    h.major_cycle(0, model[0], rho[0], gammas[0], mus[0], local_out=local)
    start = torch.tensor(np.random.default_rng(7).standard_normal((n, n)), dtype=torch.float32,
                         device="cuda")
    h.minor_cycle_fista(0, local, start, rho_other=rho[0], n_iter=2, power_iters=2, gamma_n=1.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h.minor_cycle_fista(0, local, start, rho_other=rho[0], n_iter=200, power_iters=30,
                        gamma_n=1.0)
    t_fista = time.perf_counter() - t0
    out["fista"] = {
        "ms": round(1e3 * t_fista, 2), "iterations": 200, "power_iterations": 30,
        "ms_per_iteration": round(1e3 * t_fista / 230, 3),
        "config": "node V_L, Eq. 5 with gamma_n = 1, %d^2, db8 3 levels, lambda = 1e-3 "
                  "max |i~|, FP64 transforms" % n}
    # the paper's dictionary (db1 .. db8 concatenated) and iteration count (50)
    h.minor_cycle_fista(0, local, start, rho_other=rho[0], n_iter=2, power_iters=2, gamma_n=1.0,
                        dictionary=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h.minor_cycle_fista(0, local, start, rho_other=rho[0], n_iter=50, power_iters=30,
                        gamma_n=1.0, dictionary=True)
    t_fd = time.perf_counter() - t0
    out["fista_dictionary"] = {
        "ms": round(1e3 * t_fd, 2), "iterations": 50, "power_iterations": 30,
        "config": "node V_L, Eq. 5 with gamma_n = 1, %d^2, W = the concatenation of db1 .. db8 "
                  "(8 N^2 coefficients), 3 levels, lambda = 1e-3 max |i~|, FP64 transforms" % n}
    log("minor cycles at N = %d: %s, FISTA %.1f ms (200 + 30 power), FISTA with the 8-basis "
        "dictionary %.1f ms (50 + 30 power)"
        % (n, ("msCLEAN %.1f ms (%d iterations)" % (out["msclean"]["ms"],
                                                    out["msclean"]["iterations"]))
           if "msclean" in out else "no msCLEAN", 1e3 * t_fista, 1e3 * t_fd))
    return out


def whole_loop(h, n, name):
    """Device time of the workload's whole reconstruction as configured,
    through the library's one-call loops: the 15.7M-visibility workload's
    decentralized multi-scale CLEAN (10 major cycles, S = {0, 4, 12} px,
    gain 0.1, K = 2000, threshold 1e-4) or the 50M-visibility workload's
    sparsity-regularised loop (5 major cycles of FISTA: db8, 3 levels, 200
    iterations, 30 power iterations, lambda = 1e-3 max |i~|)."""
    import numpy as np
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if name == "decentral":
        _, _, _, counts = h.reconstruct_msclean(10, [0, 4, 12], gain=0.1, niter=2000,
                                                threshold=1e-4)
        t = time.perf_counter() - t0
        out = {"ms": round(1e3 * t, 1), "major_cycles": 10,
               "components": int(np.asarray(counts).sum()),
               "config": "decentralized msCLEAN, 10 major cycles, S = {0, 4, 12} px, gain 0.1, "
                         "K = 2000, threshold 1e-4, both nodes"}
    else:
        rng = np.random.default_rng(9)
        starts = [torch.tensor(rng.standard_normal((n, n)), dtype=torch.float32, device="cuda")
                  for _ in range(2)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h.reconstruct_fista(5, starts, n_iter=200, power_iters=30)
        t = time.perf_counter() - t0
        out = {"ms": round(1e3 * t, 1), "major_cycles": 5,
               "config": "decentralized FISTA (Eq. 5), 5 major cycles, db8, 3 levels, 200 "
                         "iterations + 30 power iterations per cycle and node, lambda = 1e-3 "
                         "max |i~|, both nodes"}
    log("%s: whole reconstruction as configured, %.1f ms (%s)" % (name, out["ms"], out["config"]))
    return out


def batch_oracle(d, chans, kept, models, got, args, tag):
    """The FP64 oracle's residual image (Eq. 2) of every 8th channel, over all
    of its unflagged visibilities (oracle.pool on the host's cores), against
    the timed fused cycle's outputs; also the oracle's rate on them."""
    import numpy as np
    from oracle import geometry, imaging, pool
    workers = args.oracle_workers or pool.default_workers()
    uvw = d["uvw"].cpu().numpy() if hasattr(d["uvw"], "cpu") else d["uvw"]
    errs, n_vis, secs = {}, 0, 0.0
    for k, (vis, flag) in kept.items():
        c = chans[k]
        n = c["n_img"]
        u, v = geometry.uv_lambda(uvw, c["freq_hz"])
        valid = flag == 0
        w = imaging.uniform_weights(u, v, n, c["cell"], valid=valid)
        model = models[k].cpu().numpy().astype(np.float64)
        t0 = time.perf_counter()
        ref, _ = pool.residual_image(u[valid], v[valid], vis[valid], w[valid], model, c["cell"],
                                     workers=workers)
        secs += time.perf_counter() - t0
        n_vis += int(valid.sum())
        g = got[k].cpu().numpy().astype(np.float64)
        errs[str(k)] = float(np.linalg.norm(g - ref) / np.linalg.norm(ref))
    out = {"channels": sorted(int(k) for k in kept), "rel_l2": errs,
           "max_rel_l2": max(errs.values()), "tolerance": 1e-5,
           "pass": bool(max(errs.values()) <= 1e-5),
           "oracle_mvis_per_s": round(n_vis / secs / 1e6, 3), "oracle_seconds": round(secs, 1),
           "oracle_cores": workers}
    log("%s: oracle on every 8th channel (%d channels, %d visibilities, %d processes): %.1f s, "
        "%.3f Mvis/s; GPU error max %.2e" % (tag, len(kept), n_vis, workers, secs,
                                             out["oracle_mvis_per_s"], out["max_rel_l2"]))
    return out


def batched_channels(args, small=False):
    """Batched-channel workload: the major cycle (Eq. 2) of every channel of
    a 64-channel observation (0.95 - 1.75 GHz, 256 antennas, 480 times,
    flags 0-60 % per channel, images 512 / 1024 / 2048), one partition per
    channel; with ``small``, 256 short channels of the same array (16 times,
    images 256 / 512), where one channel's launch cannot fill the chip.
    Support from the 1e-5 accuracy rule, tile and chunk cap from the
    create-time autotuner on the largest channel, then the chunk cap re-tuned
    over the fused launch.  Times the fused batch as a replayed HIP graph,
    the same eagerly, and the per-channel launch loop."""
    import numpy as np
    import torch
    from paper_2507_22128_amd import imager, synth
    t0 = time.perf_counter()
    cfg = dict(synth.CHANNELS)
    if small:
        cfg.update(n_chan=args.batch_small_channels, n_time=16, t_min=8, sizes=(256, 512))
    else:
        cfg["n_chan"] = args.batch_channels
    d = synth.make_channels(device="cuda", **cfg)
    torch.cuda.synchronize()
    chans = d["channels"]
    n_ok = [int((c["flag"] == 0).sum().item()) for c in chans]
    tag = "batch (small channels)" if small else "batch"
    log("%s: %d channels generated in %.1f s, %d - %d unflagged visibilities per channel"
        % (tag, len(chans), time.perf_counter() - t0, min(n_ok), max(n_ok)))

    def mk(c, **kw):
        return imager.Imager.create(uvw=d["uvw"], vis=c["vis"], freq_hz=c["freq_hz"],
                                    cell=c["cell"], n_pix=c["n_img"], flag=c["flag"],
                                    n_partitions=1, weighting="uniform", **kw)

    t0 = time.perf_counter()
    first = int(np.argmax(n_ok))
    members = [None] * len(chans)
    members[first] = mk(chans[first], support=0, tolerance=1e-5, autotune=True)
    i0 = members[first].info
    tune_log = members[first].tune_log()
    for k, c in enumerate(chans):
        if members[k] is None:
            members[k] = mk(c, support=i0.support, tile=i0.tile, chunk=i0.chunk)
    create_s = time.perf_counter() - t0
    # host copies of every 8th channel, for the oracle check of the timed outputs
    sample = (list(range(0, len(chans), 8))
              if (not small and args.batch_oracle and not args.no_cpu_baseline) else [])
    kept = {k: (chans[k]["vis"].cpu().numpy(), chans[k]["flag"].cpu().numpy()) for k in sample}
    for c in chans:  # the handles hold their own copies
        c["vis"] = c["flag"] = None
    torch.cuda.empty_cache()
    b = imager.Batch(members)
    chosen, cap_ms = b.autotune()
    info = b.info()
    log("%s: %d members created in %.1f s (support %d, tile %d from the create tuner), "
        "chunk cap %d from the batch tuner %s" % (tag, len(members), create_s, i0.support, i0.tile,
                                                 chosen, cap_ms))
    g = torch.Generator(device="cuda")
    g.manual_seed(11)
    models = []
    for m in members:
        n = m.n_pix
        x = torch.zeros(n * n, device="cuda")
        idx = torch.randint(0, n * n, (200,), generator=g, device="cuda")
        x[idx] = torch.rand(200, generator=g, device="cuda")
        models.append(x.view(n, n))
    res = [torch.empty((m.n_pix, m.n_pix), device="cuda") for m in members]
    out = {}
    last = {}
    for name, mode in (("fused_graph", dict(graph=True)), ("fused_eager", {}),
                       ("per_channel_loop", dict(loop=True))):
        for _ in range(args.warmup):
            b.major_cycle(models, res, **mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.batch_steps):
            b.major_cycle(models, res, **mode)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / args.batch_steps
        out[name] = {"ms_per_cycle": round(ms, 3),
                     "mvis_per_s": round(info.n_vis / (ms / 1e3) / 1e6, 1)}
        last[name] = [r.clone() for r in res]
        log("%s %s: %.3f ms per cycle of all channels, %.0f Mvis/s"
            % (tag, name, ms, info.n_vis / (ms / 1e3) / 1e6))
    # the same fused cycle in member sets of 128 MB (half of the last-level
    # cache), each set's stages back to back (default: one set, one
    # de/gridding launch and one flush for all channels)
    n_sets = int(b.info().n_sets)
    b.set_bytes(128 << 20)
    n_sets_cache = int(b.info().n_sets)
    for name, mode in (("fused_sets_128mb_graph", dict(graph=True)),
                       ("fused_sets_128mb_eager", {})):
        for _ in range(args.warmup):
            b.major_cycle(models, res, **mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.batch_steps):
            b.major_cycle(models, res, **mode)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / args.batch_steps
        out[name] = {"ms_per_cycle": round(ms, 3),
                     "mvis_per_s": round(info.n_vis / (ms / 1e3) / 1e6, 1)}
        last[name] = [r.clone() for r in res]
        log("%s %s: %.3f ms per cycle of all channels, %.0f Mvis/s"
            % (tag, name, ms, info.n_vis / (ms / 1e3) / 1e6))
    b.set_bytes(0)
    if sample:
        out["oracle_every_8th_channel"] = batch_oracle(d, chans, kept, models, last["fused_graph"],
                                                       args, tag)
    same = all(torch.equal(a, c) for a, c in zip(last["fused_graph"], last["per_channel_loop"]))
    same = same and all(torch.equal(a, c) for a, c in zip(last["fused_graph"],
                                                          last["fused_sets_128mb_graph"]))
    sizes = [m.n_pix for m in members]
    t_win = cap_ms[chosen] / 1e3
    flops = flops_per_vis(i0.support) * info.n_vis
    out.update({
        "workload": "%d channels %.2f - %.2f GHz, %d antennas, %d baselines x T_c times with "
                    "T_c uniform in %d .. %d per channel, flags uniform 0 - %.0f %% per channel, "
                    "images %s, complex64, uniform weighting, 1 partition per channel"
                    % (len(chans), cfg["f_lo"] / 1e9, cfg["f_hi"] / 1e9, cfg["n_ant"],
                       cfg["n_ant"] * (cfg["n_ant"] - 1) // 2,
                       cfg.get("t_min") or cfg["n_time"], cfg["n_time"], 100 * cfg["flag_max"],
                       "/".join(str(x) for x in cfg["sizes"])),
        "n_channels": len(members),
        "n_vis": int(info.n_vis),
        "image_sizes": {str(x): sizes.count(x) for x in sorted(set(sizes))},
        "support": i0.support, "tile": i0.tile, "chunk": chosen,
        "n_chunks_fused": int(info.n_chunks),
        "n_sets": n_sets,
        "n_sets_128mb": n_sets_cache,
        "time_samples_per_channel": [int(min(c["n_time"] for c in chans)),
                                     int(max(c["n_time"] for c in chans))],
        "n_vis_per_channel": [int(min(n_ok)), int(max(n_ok))],
        "create_tuner": [{"tile": t, "chunk": c, "ms": round(x, 4)} for t, c, x in tune_log],
        "batch_tuner_ms": {str(k): round(v, 4) for k, v in cap_ms.items()},
        "fused_window_flush_ms": round(cap_ms[chosen], 4),
        "fused_window_flush_tflops": round(flops / t_win / 1e12, 2),
        "speedup_graph_vs_loop": round(out["per_channel_loop"]["ms_per_cycle"]
                                       / out["fused_graph"]["ms_per_cycle"], 3),
        "graph_equals_loop_bitwise": bool(same),
        "create_s": round(create_s, 1),
    })
    b.destroy()
    for m in members:
        m.destroy()
    del d
    torch.cuda.empty_cache()
    return out


def serving(args):
    """Serving workload: a Poisson stream of imaging requests shaped like the
    single-channel workloads (the 256-antenna array, 1 - 50M visibilities
    log-uniform, images 512 / 1024 / 2048, msCLEAN (S = {0, 4, 12}) or
    FISTA (db8), 1 or 2 partitions, 5 - 10 major cycles), served with
    admission by device-memory footprint and continuous batching at cycle
    boundaries, at each arrival rate; compared with plain serial execution
    of the same requests."""
    import numpy as np
    import torch
    from paper_2507_22128_amd import serve, synth
    n_req = args.serve_requests
    t0 = time.perf_counter()
    d = synth.make_requests(n_req, seed=6, device="cuda")
    torch.cuda.synchronize()
    log("serving: %d requests generated in %.1f s (%.1f - %.1f M visibilities, images %s)"
        % (n_req, time.perf_counter() - t0, min(r["n_vis"] for r in d) / 1e6,
           max(r["n_vis"] for r in d) / 1e6, sorted(set(r["n_img"] for r in d))))
    rng = np.random.default_rng(8)
    reqs = []
    for k, r in enumerate(d):
        reqs.append(serve.Request(
            uvw=r["uvw"], vis=r["vis"], freq_hz=r["freq_hz"], cell=r["cell"], n_pix=r["n_img"],
            method="msclean" if rng.random() < 0.5 else "fista",
            n_cycles=int(rng.integers(5, 11)), n_partitions=int(rng.integers(1, 3)),
            niter=args.serve_clean_iter, fista_iter=args.serve_fista_iter,
            power_iters=args.serve_power_iter, name="req%d" % k, power_seed=k))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    serial = serve.run_serial(reqs)
    t_serial = time.perf_counter() - t0
    ref = [f for f, _ in serial]
    service = [t for _, t in serial]
    log("serving: %d requests, plain serial execution %.2f s" % (n_req, t_serial))
    out = {"requests": n_req,
           "mix": {"msclean": sum(r.method == "msclean" for r in reqs),
                   "fista": sum(r.method == "fista" for r in reqs),
                   "two_partitions": sum(r.n_partitions == 2 for r in reqs),
                   "image_sizes": {str(x): sum(r.n_pix == x for r in reqs)
                                   for x in sorted(set(r.n_pix for r in reqs))},
                   "n_vis_millions": [round(min(r.n_vis for r in reqs) / 1e6, 2),
                                      round(max(r.n_vis for r in reqs) / 1e6, 2)],
                   "cycles": [int(min(r.n_cycles for r in reqs)),
                              int(max(r.n_cycles for r in reqs))],
                   "per_cycle": "msCLEAN K = %d per node, FISTA %d iterations + %d power "
                                "iterations" % (args.serve_clean_iter, args.serve_fista_iter,
                                                args.serve_power_iter)},
           "hbm_budget_gib": args.serve_budget_gib, "workers": args.serve_workers,
           "rates": {}}
    vis_cycles = None
    for rate in args.serve_rates:
        arr = np.cumsum(np.random.default_rng(int(rate * 1000)).exponential(1.0 / rate, n_req))
        with serve.Server(hbm_budget=int(args.serve_budget_gib * 2 ** 30),
                          workers=args.serve_workers) as srv:
            t0 = time.perf_counter()
            futs = []
            for req, at in zip(reqs, arr):
                dt = t0 + at - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
                futs.append(srv.submit(req))
            res = [f.result(timeout=600) for f in futs]
        makespan = max(r.finished for r in res) - t0
        vis_cycles = sum(r.n_valid * r.n_cycles for r in res)
        lat = np.array(sorted(r.latency for r in res)) * 1e3
        errs = []
        same = True
        for r, f in zip(res, ref):
            same = same and bool(torch.equal(r.final, f))
            errs.append(float(torch.linalg.norm(r.final - f) / torch.linalg.norm(f)))
        # the plain path at the same arrivals: one request after another in
        # arrival order, each taking its measured serial service time
        done, ser_lat = 0.0, []
        for at, sv in zip(arr, service):
            done = max(done, at) + sv
            ser_lat.append(done - at)
        ser_lat = np.array(sorted(ser_lat)) * 1e3
        out["rates"][str(rate)] = {
            "p50_ms": round(float(np.percentile(lat, 50)), 1),
            "p99_ms": round(float(np.percentile(lat, 99)), 1),
            "serial_p50_ms": round(float(np.percentile(ser_lat, 50)), 1),
            "serial_p99_ms": round(float(np.percentile(ser_lat, 99)), 1),
            "serial_makespan_s": round(float(done), 3),
            "makespan_s": round(makespan, 3),
            "aggregate_mvis_per_s": round(vis_cycles / makespan / 1e6, 1),
            "max_resident_requests": srv.max_resident_jobs,
            "max_concurrent_cycles": srv.max_concurrent_cycles,
            "admission_waits": srv.admission_waits,
            "max_reserved_gib": round(srv.max_reserved / 2 ** 30, 2),
            "max_rel_err_vs_serial": max(errs),
            "identical_to_serial": same,
        }
        log("serving at %.0f req/s: p50 %.0f ms, p99 %.0f ms (serial at these arrivals: %.0f / "
            "%.0f ms), makespan %.2f s, %.0f Mvis/s (serial %.0f Mvis/s), identical %s"
            % (rate, np.percentile(lat, 50), np.percentile(lat, 99), np.percentile(ser_lat, 50),
               np.percentile(ser_lat, 99), makespan, vis_cycles / makespan / 1e6,
               vis_cycles / t_serial / 1e6, same))
    out["serial"] = {"seconds": round(t_serial, 3),
                     "aggregate_mvis_per_s": round(vis_cycles / t_serial / 1e6, 1)}
    out["vis_cycles"] = int(vis_cycles)
    del d, reqs, serial, ref
    torch.cuda.empty_cache()
    return out


CONFIG_TEXT = {
    "decentral": "256 antennas in an 8 km disk, 32640 baselines x 480 times = %d visibilities "
                 "(complex64), 1 channel at 1.40 GHz, uniform weighting, 2 partitions split at "
                 "the median |uv| (delta 1 px), 1024^2 image, 2x padded grid, ES support 8; sky "
                 "200 points + 30 Gaussians (sigma 2-8 px)",
    "convex": "256 antennas in an 8 km disk, 32640 baselines x 1532 times = %d visibilities "
              "(complex64), 1 channel at 1.40 GHz, uniform weighting, 2 partitions split at the "
              "median |uv| (delta 1 px), 2048^2 image, 2x padded grid, ES support 8; sky 500 "
              "points + 50 Gaussians (sigma 4-40 px)",
}


def measure_tiny(args, with_oracle=True):
    """The plain method's small workload (one partition: 64 antennas,
    120,960 visibilities, 256^2 image, 512^2 grid).  Its cycle (Eq. 2) fits
    in the caches, so it is reported as latency: the cycle time over the
    timed steps, p50 / p99 of event-timed cycles and the per-stage times,
    with the error of the output against the oracle's residual image."""
    import numpy as np
    import torch
    from paper_2507_22128_amd import imager, synth

    d = synth.make("tiny", device="cuda")
    n = d["n_img"]
    h = imager.Imager.create(d, n_partitions=1, weighting="uniform")
    info = h.info
    model = torch.tensor(np.ascontiguousarray(0.5 * d["truth"]), dtype=torch.float32,
                         device="cuda")
    out = torch.empty((n, n), device="cuda")

    def step():
        h.major_cycle(0, model, out=out)

    # a cycle takes tens of microseconds: ten times the steps of the large
    # workloads, so that p99 is not just the slowest of a few
    steps, warmup = 10 * args.steps, 10 * args.warmup
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    got = out.cpu().numpy().astype(np.float64)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    for k in range(steps):
        ev[k][0].record()
        step()
        ev[k][1].record()
    torch.cuda.synchronize()
    per_step = sorted(a.elapsed_time(b) for a, b in ev)
    h.set_timing(True)
    for _ in range(steps):
        step()
    cycles, stage_ms = h.get_timing()
    h.set_timing(False)
    h.destroy()
    res = {
        "config": {"workload": "tiny: 64 antennas in a 2 km disk, 2016 baselines x 60 times = "
                               "%d visibilities, 1 channel at 1.40 GHz, uniform weighting, one "
                               "partition, 256^2 image, 2x padded grid, ES support 8; sky 20 "
                               "points + 3 Gaussians" % len(d["vis"]),
                   "n_vis": int(info.n_valid), "n_pix": n, "n_grid": info.n_grid},
        "ms_per_cycle": round(ms, 4),
        "p50_ms": round(per_step[len(per_step) // 2], 4),
        "p99_ms": round(per_step[min(len(per_step) - 1, int(0.99 * len(per_step)))], 4),
        "event_timed_steps": len(per_step),
        "stage_ms": {k: round(v / cycles, 4) for k, v in stage_ms.items()},
        "mvis_per_s": round(info.n_valid / (ms / 1e3) / 1e6, 1),
        "note": "cache-resident: reported as latency, not as a fraction of HBM",
    }
    if with_oracle:
        from oracle import geometry, imaging
        u, v = geometry.uv_lambda(d["uvw"], d["freq_hz"])
        w = imaging.uniform_weights(u, v, n, d["cell"])
        ref, _ = imaging.residual_image(u, v, d["vis"], w, 0.5 * d["truth"], d["cell"])
        e = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        res["err_vs_oracle"] = {"rel_l2": e, "tolerance": 1e-5, "pass": bool(e <= 1e-5)}
    log("tiny: %.4f ms per cycle (p50 %.4f, p99 %.4f ms)%s"
        % (res["ms_per_cycle"], res["p50_ms"], res["p99_ms"],
           ", error %.2e" % res["err_vs_oracle"]["rel_l2"] if with_oracle else ""))
    return res


def measure_cycle(name, args, workers, with_oracle=True, minor=True):
    """Times the decentralized major cycle of workload ``name``: both nodes'
    cycles (Eq. 2 then Eq. 7) with the model 0.5 x the true sky and the
    aggregate 0.01 x the true sky, gamma / mu from the partitions' summed
    weights.  Returns the measurement dict (value, p50 / p99, stages,
    roofline of the window kernel, errors against the oracle, minor
    cycles)."""
    import numpy as np
    import torch
    from paper_2507_22128_amd import imager, synth

    t0 = time.perf_counter()
    d = synth.make(name, device="cuda")
    n = d["n_img"]
    log("workload %s: %d visibilities, N=%d (generated in %.1f s)"
        % (name, len(d["vis"]), n, time.perf_counter() - t0))
    h = imager.Imager.create(d, n_partitions=2, weighting="uniform")
    info = h.info
    log("create: %.1f ms, partitions %d / %d visibilities, %d / %d chunks, ell %.3f px"
        % (info.create_ms, info.n_vis[0], info.n_vis[1], info.n_chunks[0], info.n_chunks[1],
           info.ell_pix))
    dev = lambda x: torch.tensor(np.ascontiguousarray(x), dtype=torch.float32, device="cuda")
    model = [dev(0.5 * d["truth"]), dev(0.5 * d["truth"])]
    rho = [dev(0.01 * d["truth"]), dev(0.01 * d["truth"])]
    out = [torch.empty((n, n), device="cuda") for _ in range(2)]
    local = [torch.empty((n, n), device="cuda") for _ in range(2)]
    wsum = [info.sum_w[0], info.sum_w[1]]
    gammas = [wsum[p] / (wsum[0] + wsum[1]) for p in (0, 1)]
    mus = [wsum[1 - p] / (wsum[0] + wsum[1]) for p in (0, 1)]

    def step():
        # both nodes' major cycles, concurrent on the device
        h.major_cycle_nodes(model, rho, gammas, mus, outs=out, local_outs=local)

    for _ in range(args.warmup):
        step()
    # the timed steps: nothing but the steps between the two synchronizations
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    outs_np = [o.cpu().numpy() for o in out]
    locs_np = [o.cpu().numpy() for o in local]
    # the same number of steps again with an event pair around each (p50 / p99
    # of the per-step device time), then with the handle's stage events (per
    # stage); both add event packets to the streams, so neither is part of the
    # timed steps
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    for k in range(args.steps):
        ev[k][0].record()
        step()
        ev[k][1].record()
    torch.cuda.synchronize()
    per_step = sorted(a.elapsed_time(b) for a, b in ev)
    h.set_timing(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    cycles, stage_ms = h.get_timing()
    stage_conc = {k: v / cycles for k, v in stage_ms.items()}
    # the same cycles one node at a time on the handle's stream: each kernel's
    # own launch duration (what a kernel trace reports), for the roofline
    for _ in range(args.steps):
        for p in (0, 1):
            h.major_cycle(p, model[p], rho[p], gammas[p], mus[p], out=out[p], local_out=local[p])
    cycles_s, stage_ms_s = h.get_timing()
    h.set_timing(False)
    stage_avg = {k: v / cycles_s for k, v in stage_ms_s.items()}
    ms_per_step = 1e3 * wall / args.steps
    value = info.n_valid / (ms_per_step / 1e3) / 1e6
    log("%s: %d steps: %.4f ms/step, %.0f Mvis/s (p50 %.4f ms, p99 %.4f ms)"
        % (name, args.steps, ms_per_step, value, per_step[len(per_step) // 2],
           per_step[min(len(per_step) - 1, int(0.99 * len(per_step)))]))
    log("%s: per node-cycle stage ms, nodes concurrent: %s" % (name, json.dumps(
        {k: round(v, 4) for k, v in stage_conc.items()})))
    log("%s: per node-cycle stage ms, one node at a time: %s" % (name, json.dumps(
        {k: round(v, 4) for k, v in stage_avg.items()})))

    # roofline of the dominant kernel, the fused de/grid window kernel: one
    # launch per node-cycle, timed by the handle's stage events on its stream
    # in the one-node-at-a-time pass; units averaged over the two launches
    ng = info.n_grid
    wt = info.support
    m_avg = 0.5 * (info.n_vis[0] + info.n_vis[1])
    t_launch = stage_avg["degrid_grid"] / 1e3
    flops = flops_per_vis(wt) * m_avg
    bytes_alg = 20.0 * m_avg
    achieved_tf = flops / t_launch / 1e12
    achieved_gbs = bytes_alg / t_launch / 1e9
    roofline = {
        "bound": "mfma",
        "achieved": round(achieved_tf, 3),
        "peak": FP32_PEAK_MATRIX,
        "unit": "TFLOP/s",
        "frac": round(achieved_tf / FP32_PEAK_MATRIX, 4),
        "traffic": measured_traffic(name),
        "kernel": "k_window<%d,%d,MODE_DEGRID_GRID> (fused degrid / residual / grid)"
                  % (wt, info.tile),
        "avg_launch_ms": round(stage_avg["degrid_grid"], 4),
        "flop_per_vis": flops_per_vis(wt),
        "vis_per_launch": m_avg,
        "hbm_achieved_gbs": round(achieved_gbs, 1),
        "hbm_frac": round(achieved_gbs / HBM_PEAK_GBS, 4),
        "bytes_alg_per_launch": bytes_alg,
    }
    # whole-cycle algorithmic bytes: visibility stream, ~8 grid passes, images
    cycle_bytes = sum(20.0 * info.n_vis[p] + 64.0 * ng * ng + 8.0 * n * n for p in (0, 1))
    res = {
        "value": round(value, 1),
        "ms_per_step": round(ms_per_step, 4),
        "config": {
            "workload": name + ": " + CONFIG_TEXT[name] % len(d["vis"]),
            "n_vis": int(info.n_valid),
            "n_vis_partitions": [int(info.n_vis[0]), int(info.n_vis[1])],
            "n_pix": n,
            "n_grid": ng,
            "parallelism": "single GPU, both partitions on one device",
        },
        "p50_ms": round(per_step[len(per_step) // 2], 4),
        "p99_ms": round(per_step[min(len(per_step) - 1, int(0.99 * len(per_step)))], 4),
        "event_timed_steps": len(per_step),
        "create_ms": round(info.create_ms, 1),
        "stage_ms_per_node_cycle": {k: round(v, 4) for k, v in stage_avg.items()},
        "stage_ms_per_node_cycle_concurrent": {k: round(v, 4) for k, v in stage_conc.items()},
        "cycle_hbm_frac": round(cycle_bytes / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        # the partitions' members summed (visibilities of the overlap ring counted in both)
        "mvis_per_s_partition_sum": round((info.n_vis[0] + info.n_vis[1]) /
                                          (ms_per_step / 1e3) / 1e6, 1),
        # the fused degrid / residual / grid kernel alone, one launch per partition
        "degrid_grid_kernel_mvis_per_s": round(m_avg / t_launch / 1e6, 1),
        "roofline": roofline,
    }
    if minor:
        res["minor_cycles"] = minor_cycles(h, info, model, rho, gammas, mus, n,
                                           msclean=(name == "decentral"))
        if not args.no_reconstruction:
            res["reconstruction"] = whole_loop(h, n, name)
    h.destroy()
    del model, rho, out, local
    torch.cuda.empty_cache()
    if with_oracle:
        log("%s: oracle on the full partitions (%d processes) ..." % (name, workers))
        base, err = oracle_cycle(d, outs_np, locs_np, workers)
        res["err_vs_oracle"] = err
        res["cpu_baseline"] = base
        log("%s: oracle %.1f s (%.3f Mvis/s); GPU error vs oracle: composed %s, local %s"
            % (name, base["seconds"], base["value"],
               ["%.2e" % e for e in err["composed_rel_l2"]],
               ["%.2e" % e for e in err["local_rel_l2"]]))
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="convex")
    ap.add_argument("--oracle-workers", type=int, default=0,
                    help="host processes of the oracle run (0: every core this process may use)")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle run (no cpu_baseline, no error against the oracle)")
    ap.add_argument("--no-minor-cycles", action="store_true")
    ap.add_argument("--no-reconstruction", action="store_true",
                    help="skip the whole reconstructions as configured (the one-call loops)")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-decentral", action="store_true")
    ap.add_argument("--no-tiny", action="store_true",
                    help="skip the latency of the one-partition 120,960-visibility cycle")
    ap.add_argument("--batch-channels", type=int, default=64)
    ap.add_argument("--batch-small-channels", type=int, default=256)
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--no-batch-oracle", dest="batch_oracle", action="store_false",
                    help="skip the oracle check of every 8th batched channel")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=50)
    ap.add_argument("--serve-rates", type=float, nargs="+", default=[2.0, 5.0, 10.0, 20.0, 50.0])
    ap.add_argument("--serve-workers", type=int, default=4)
    ap.add_argument("--serve-budget-gib", type=float, default=64.0)
    ap.add_argument("--serve-clean-iter", type=int, default=200)
    ap.add_argument("--serve-fista-iter", type=int, default=20)
    ap.add_argument("--serve-power-iter", type=int, default=10)
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="before the steps, run a plain device copy of this many MiB three "
                         "times (a known-size kernel to scale hardware byte counters by)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the imager runs on a single GPU; --gpus %d is not supported "
              "(the two partitions run on one device)" % max(args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import torch
    from oracle import pool
    workers = args.oracle_workers or pool.default_workers()

    if args.calibrate_copy_mb:
        nb = args.calibrate_copy_mb << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: 3 x %d MiB device to device" % args.calibrate_copy_mb)
        del src, dst

    head = measure_cycle(args.workload, args, workers, with_oracle=not args.no_cpu_baseline,
                         minor=not args.no_minor_cycles)
    res = {
        "metric": METRIC,
        "value": head.pop("value"),
        "unit": "Mvis/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": head.pop("config"),
    }
    res.update(head)
    if args.workload != "decentral" and not args.no_decentral:
        res["decentral"] = measure_cycle("decentral", args, workers,
                                         with_oracle=not args.no_cpu_baseline,
                                         minor=not args.no_minor_cycles)
    if not args.no_tiny:
        res["tiny"] = measure_tiny(args, with_oracle=not args.no_cpu_baseline)
    if not args.no_batch:
        res["batched_channels"] = batched_channels(args)
        res["batched_small_channels"] = batched_channels(args, small=True)
    if not args.no_serve:
        res["serving"] = serving(args)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
