"""Sparsity-regularised minor cycle (FISTA, db8 wavelets) on the GPU against
the FP64 oracle (GPU required).

Teacher forcing: both sides get the same residual image and PSF (made by
the oracle, rounded to float32), aggregate rho and power-iteration start
(seeded), then run the same number of power and FISTA iterations.  The GPU evaluates H and
Gamma with FP32 transforms and keeps the coefficients in FP64; the bar is a
relative L2 error of 1e-6 on the deconvolved image (its float32 rounding
is about 3e-8) and 1e-10 on L_hat, lambda and the objective; the
transforms run in FP64 because FISTA's momentum amplifies operator
rounding over hundreds of iterations.
"""

import numpy as np
import pytest

from helpers import (f32, imaging, oracle_inputs, oracle_weights, rel, say, to_dev, to_np, uv,
                     workload)

pytestmark = pytest.mark.gpu


def _imager():
    from paper_2507_22128_amd import imager
    return imager


@pytest.fixture(scope="module")
def tiny1():
    say("case: tiny workload, 1 partition (FISTA)")
    d = workload("tiny")
    h = _imager().Imager.create(d, n_partitions=1, weighting="uniform")
    yield d, h
    h.destroy()


@pytest.fixture(scope="module")
def tiny2():
    say("case: tiny workload (20 time steps), 2 partitions (FISTA)")
    d = workload("tiny", n_time=20)
    h = _imager().Imager.create(d, n_partitions=2, weighting="uniform")
    yield d, h
    h.destroy()


def _oracle_run(dirty, psf, rho, gamma_n, ell, delta, own, start, n_iter, power_iters, serial,
                lam_frac=1e-3, dictionary=False):
    from oracle import fista, wavelets
    h = [wavelets.daubechies(p) for p in range(1, 9)] if dictionary else wavelets.daubechies(8)
    prob = fista.NodeProblem(dirty, psf, rho, gamma_n, ell, delta, own, h, 3, serial=serial)
    L = fista.power_iteration(prob, start, power_iters)
    lam = lam_frac * np.abs(dirty).max()
    alpha, obj = fista.fista(prob, lam, n_iter, L)
    return prob.W(alpha), np.array(obj), L, lam


def _serial_inputs():
    o = oracle_inputs("tiny")
    return f32(o["resid"][0]), f32(o["psf"][0])


def test_fista_serial_teacher_forced(tiny1):
    d, h = tiny1
    n = d["n_img"]
    dirty, psf = _serial_inputs()
    start = f32(np.random.default_rng(31).standard_normal((n, n)))
    delta, obj, L, lam = h.minor_cycle_fista(0, to_dev(dirty), to_dev(start), psf=to_dev(psf),
                                             n_iter=200, power_iters=30, serial=True,
                                             want_objective=True)
    r_img, r_obj, r_L, r_lam = _oracle_run(dirty, psf, None, 0.0, 0.0, 1.0, "L", start, 200, 30,
                                           serial=True)
    e_img, e_obj = rel(to_np(delta), r_img), np.abs(obj / r_obj - 1).max()
    say("serial FISTA: L %.6g (oracle %.6g), lambda %.4g, image rel err %.3e, objective rel %.3e"
        % (L, r_L, lam, e_img, e_obj))
    assert abs(L / r_L - 1) < 1e-10 and abs(lam / r_lam - 1) < 1e-10
    assert e_obj < 1e-10
    assert e_img < 1e-6


def test_fista_dictionary_teacher_forced(tiny1, tiny2):
    """W = the concatenation of db1 .. db8 (the paper's dictionary), serial and
    node H of the decentralized problem, 80 iterations."""
    d, h = tiny1
    n = d["n_img"]
    dirty, psf = _serial_inputs()
    start = f32(np.random.default_rng(41).standard_normal((n, n)))
    delta, obj, L, lam = h.minor_cycle_fista(0, to_dev(dirty), to_dev(start), psf=to_dev(psf),
                                             n_iter=80, power_iters=20, serial=True,
                                             want_objective=True, dictionary=True)
    r_img, r_obj, r_L, r_lam = _oracle_run(dirty, psf, None, 0.0, 0.0, 1.0, "L", start, 80, 20,
                                           serial=True, dictionary=True)
    e_img, e_obj = rel(to_np(delta), r_img), np.abs(obj / r_obj - 1).max()
    say("dictionary FISTA (serial): L %.6g (oracle %.6g), image rel err %.3e, objective rel %.3e"
        % (L, r_L, e_img, e_obj))
    assert abs(L / r_L - 1) < 1e-10 and abs(lam / r_lam - 1) < 1e-10
    assert e_obj < 1e-10 and e_img < 1e-6
    d2, h2 = tiny2
    rng = np.random.default_rng(42)
    o = oracle_inputs("tiny", n_time=20, partitions=2, model_scale=0.3)
    assert h2.info.ell_pix == o["ell"] and h2.info.delta_pix == 1.0
    rho = f32(0.002 * rng.standard_normal((n, n)))
    local, psf2 = f32(o["resid"][1]), f32(o["psf"][1])
    delta, obj, L, lam = h2.minor_cycle_fista(1, to_dev(local), to_dev(start), psf=to_dev(psf2),
                                              rho_other=to_dev(rho), n_iter=60, power_iters=20,
                                              gamma_n=1.0, want_objective=True, dictionary=True)
    r_img, r_obj, r_L, r_lam = _oracle_run(local, psf2, rho, 1.0, o["ell"], 1.0, "H", start, 60,
                                           20, serial=False, dictionary=True)
    e_img, e_obj = rel(to_np(delta), r_img), np.abs(obj / r_obj - 1).max()
    say("dictionary FISTA (node H, Eq. 5): image rel err %.3e, objective rel %.3e" % (e_img, e_obj))
    assert abs(L / r_L - 1) < 1e-10
    assert e_obj < 1e-10 and e_img < 1e-6


def test_fista_two_nodes_teacher_forced(tiny2):
    d, h = tiny2
    n = d["n_img"]
    rng = np.random.default_rng(32)
    o = oracle_inputs("tiny", n_time=20, partitions=2, model_scale=0.3)
    assert h.info.ell_pix == o["ell"] and h.info.delta_pix == 1.0
    rho = f32(0.002 * rng.standard_normal((n, n)))
    for p, own in ((0, "L"), (1, "H")):
        local, psf = f32(o["resid"][p]), f32(o["psf"][p])
        start = f32(rng.standard_normal((n, n)))
        delta, obj, L, lam = h.minor_cycle_fista(p, to_dev(local), to_dev(start), psf=to_dev(psf),
                                                 rho_other=to_dev(rho), n_iter=40,
                                                 power_iters=20, gamma_n=1.0, want_objective=True)
        r_img, r_obj, r_L, r_lam = _oracle_run(local, psf, rho, 1.0, o["ell"], 1.0, own, start,
                                               40, 20, serial=False)
        e_img, e_obj = rel(to_np(delta), r_img), np.abs(obj / r_obj - 1).max()
        say("node %s FISTA: L %.6g (oracle %.6g), image rel err %.3e, objective rel %.3e"
            % (own, L, r_L, e_img, e_obj))
        assert abs(L / r_L - 1) < 1e-10 and abs(lam / r_lam - 1) < 1e-10
        assert e_obj < 1e-10
        assert e_img < 1e-6


def test_reconstruct_fista_end_to_end(tiny2):
    d, h = tiny2
    from oracle import decentral
    n = d["n_img"]
    u, v = uv(d)
    w = oracle_weights(d, n)
    rng = np.random.default_rng(33)
    starts = {"L": rng.standard_normal((n, n)), "H": rng.standard_normal((n, n))}
    final, models, rhos, Ls, lams = h.reconstruct_fista(
        2, [to_dev(starts["L"]), to_dev(starts["H"])], n_iter=25, power_iters=15)
    ref_final, ref_models, hist = decentral.reconstruct_fista(
        u, v, d["vis"], w, n, d["cell"], 2,
        {k: f32(s) for k, s in starts.items()}, n_iter=25,
        power_iters=15, partitions=2)
    err = rel(to_np(final), ref_final)
    say("FISTA end-to-end: final rel err %.3e, L_hat %s" % (err, Ls.tolist()))
    for c, hc in enumerate(hist):
        for k, node in enumerate(("L", "H")):
            assert abs(Ls[c, k] / hc[node][1] - 1) < 1e-5
            # lambda = 1e-3 max |i~|: after the first cycle the residual
            # cancels, so its error is measured against the first cycle's
            # lambda (the dirty image's scale)
            assert abs(lams[c, k] - hc[node][0]) < 1e-5 * hist[0][node][0]
    assert err < 1e-5


@pytest.mark.timeout(900)
def test_fista_at_the_2048_workload_teacher_forced():
    """FISTA as the 50M-visibility 2048^2 workload configures it (db8, 3
    levels, lambda = 1e-3 max |i~|, 30 power iterations; Eq. 5 with gamma_n
    = 1 on node V_L), teacher-forced at that size: the node's local residual
    of 0.5 x truth and its PSF made by the oracle over the whole partition
    (25.1M visibilities, oracle.pool on the host's cores), rho = 0.01 x
    truth.  10 FISTA iterations: each of the oracle's wavelet transforms and
    PSF convolutions takes seconds at 2048^2, and the GPU runs the same
    kernels whatever the count."""
    import scipy.fft
    from oracle import pool
    from paper_2507_22128_amd import synth
    say("case: FISTA at N = 2048 (50,004,480 visibilities, node V_L), 30 power + 10 iterations")
    d = synth.make("convex", device="cuda")
    n = d["n_img"]
    u, v = uv(d)
    w = imaging.uniform_weights(u, v, n, d["cell"])
    low, _, ell = imaging.partition(u, v, n, d["cell"])
    workers = pool.default_workers()
    local = f32(pool.residual_image(u[low], v[low], d["vis"][low], w[low], 0.5 * d["truth"],
                                    d["cell"], workers=workers)[0])
    psf = f32(pool.psf2(u[low], v[low], w[low], n, d["cell"], workers=workers))
    rho = f32(0.01 * d["truth"])
    start = f32(np.random.default_rng(34).standard_normal((n, n)))
    h = _imager().Imager.create(d, n_partitions=2, weighting="uniform")
    try:
        assert h.info.ell_pix == ell and h.info.delta_pix == 1.0
        delta, obj, L, lam = h.minor_cycle_fista(0, to_dev(local), to_dev(start), psf=to_dev(psf),
                                                 rho_other=to_dev(rho), n_iter=10,
                                                 power_iters=30, gamma_n=1.0, want_objective=True)
        got = to_np(delta)
    finally:
        h.destroy()
    with scipy.fft.set_workers(workers):
        r_img, r_obj, r_L, r_lam = _oracle_run(local, psf, rho, 1.0, ell, 1.0, "L", start, 10, 30,
                                               serial=False)
    e_img, e_obj = rel(got, r_img), np.abs(obj / r_obj - 1).max()
    say("N = 2048 FISTA: L %.6g (oracle %.6g), lambda %.4g, image rel err %.3e, objective rel "
        "%.3e" % (L, r_L, lam, e_img, e_obj))
    assert abs(L / r_L - 1) < 1e-10 and abs(lam / r_lam - 1) < 1e-10
    assert e_obj < 1e-10
    assert e_img < 1e-6


@pytest.mark.parametrize("vanishing,levels", [(2, 5), (1, 6), (10, 2)])
def test_fista_smallest_image_deepest_levels(vanishing, levels):
    """N = 64, the smallest image: the wavelet levels down to 2 x 2 blocks
    (db2 over 5 levels, db1 over 6) and the 20-tap db10 over 32 x 32 blocks,
    where the filters wrap around a block more than once; serial FISTA (Eq. 4)
    on the oracle's dirty image and PSF, against the oracle."""
    from oracle import fista, wavelets
    d = workload("tiny", n_time=8)
    n = 64
    u, v = uv(d)
    w = imaging.uniform_weights(u, v, n, d["cell"])
    dirty = f32(imaging.dirty_image(u, v, d["vis"], w, n, d["cell"]))
    psf = f32(imaging.psf2(u, v, w, n, d["cell"]))
    start = f32(np.random.default_rng(35).standard_normal((n, n)))
    h = _imager().Imager.create(d, n_pix=n, n_partitions=1, weighting="uniform")
    try:
        delta, obj, L, lam = h.minor_cycle_fista(0, to_dev(dirty), to_dev(start), psf=to_dev(psf),
                                                 n_iter=60, power_iters=20, serial=True,
                                                 vanishing=vanishing, levels=levels,
                                                 want_objective=True)
        got = to_np(delta)
    finally:
        h.destroy()
    prob = fista.NodeProblem(dirty, psf, None, 0.0, 0.0, 1.0, "L",
                             wavelets.daubechies(vanishing), levels, serial=True)
    r_L = fista.power_iteration(prob, start, 20)
    r_lam = 1e-3 * np.abs(dirty).max()
    alpha, r_obj = fista.fista(prob, r_lam, 60, r_L)
    e_img, e_obj = rel(got, prob.W(alpha)), np.abs(obj / np.array(r_obj) - 1).max()
    say("N = 64, db%d, %d levels: L %.6g (oracle %.6g), image rel err %.3e, objective rel %.3e"
        % (vanishing, levels, L, r_L, e_img, e_obj))
    assert abs(L / r_L - 1) < 1e-10 and abs(lam / r_lam - 1) < 1e-10
    assert e_obj < 1e-10 and e_img < 1e-6
