"""Sparsity-regularised minor cycle (FISTA, db8 wavelets) on the GPU against
the FP64 oracle (GPU required).

Teacher forcing: both sides get the same residual image, PSF, aggregate rho
and power-iteration start (the GPU's float32 arrays, up-cast exactly), then
run the same number of power and FISTA iterations.  The GPU evaluates H and
Gamma with FP32 transforms and keeps the coefficients in FP64; the bar is a
relative L2 error of 1e-6 on the deconvolved image (its float32 rounding
is about 3e-8) and 1e-10 on L_hat, lambda and the objective; the
transforms run in FP64 because FISTA's momentum amplifies operator
rounding over hundreds of iterations.
"""

import numpy as np
import pytest

from helpers import oracle_weights, rel, say, to_dev, to_np, uv, workload

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


def test_fista_serial_teacher_forced(tiny1):
    import torch
    d, h = tiny1
    n = d["n_img"]
    dirty = h.major_cycle(0, torch.zeros((n, n), device="cuda"))
    psf = h.psf(0)
    start = to_dev(np.random.default_rng(31).standard_normal((n, n)))
    delta, obj, L, lam = h.minor_cycle_fista(0, dirty, start, n_iter=200, power_iters=30,
                                             serial=True, want_objective=True)
    r_img, r_obj, r_L, r_lam = _oracle_run(
        to_np(dirty).astype(np.float64), to_np(psf).astype(np.float64), None, 0.0, 0.0, 1.0, "L",
        to_np(start).astype(np.float64), 200, 30, serial=True)
    e_img, e_obj = rel(to_np(delta), r_img), np.abs(obj / r_obj - 1).max()
    say("serial FISTA: L %.6g (oracle %.6g), lambda %.4g, image rel err %.3e, objective rel %.3e"
        % (L, r_L, lam, e_img, e_obj))
    assert abs(L / r_L - 1) < 1e-10 and abs(lam / r_lam - 1) < 1e-10
    assert e_obj < 1e-10
    assert e_img < 1e-6


def test_fista_dictionary_teacher_forced(tiny1, tiny2):
    """W = the concatenation of db1 .. db8 (the paper's dictionary), serial and
    node H of the decentralized problem, 80 iterations."""
    import torch
    d, h = tiny1
    n = d["n_img"]
    dirty = h.major_cycle(0, torch.zeros((n, n), device="cuda"))
    psf = h.psf(0)
    start = to_dev(np.random.default_rng(41).standard_normal((n, n)))
    delta, obj, L, lam = h.minor_cycle_fista(0, dirty, start, n_iter=80, power_iters=20,
                                             serial=True, want_objective=True, dictionary=True)
    r_img, r_obj, r_L, r_lam = _oracle_run(
        to_np(dirty).astype(np.float64), to_np(psf).astype(np.float64), None, 0.0, 0.0, 1.0, "L",
        to_np(start).astype(np.float64), 80, 20, serial=True, dictionary=True)
    e_img, e_obj = rel(to_np(delta), r_img), np.abs(obj / r_obj - 1).max()
    say("dictionary FISTA (serial): L %.6g (oracle %.6g), image rel err %.3e, objective rel %.3e"
        % (L, r_L, e_img, e_obj))
    assert abs(L / r_L - 1) < 1e-10 and abs(lam / r_lam - 1) < 1e-10
    assert e_obj < 1e-10 and e_img < 1e-6
    d2, h2 = tiny2
    rng = np.random.default_rng(42)
    model = to_dev(0.3 * d2["truth"])
    rho = to_dev(0.002 * rng.standard_normal((n, n)))
    local = torch.empty((n, n), device="cuda")
    h2.major_cycle(1, model, out=torch.empty((n, n), device="cuda"), local_out=local)
    psf2 = h2.psf(1)
    delta, obj, L, lam = h2.minor_cycle_fista(1, local, start, rho_other=rho, n_iter=60,
                                              power_iters=20, gamma_n=1.0, want_objective=True,
                                              dictionary=True)
    r_img, r_obj, r_L, r_lam = _oracle_run(
        to_np(local).astype(np.float64), to_np(psf2).astype(np.float64),
        to_np(rho).astype(np.float64), 1.0, h2.info.ell_pix, h2.info.delta_pix, "H",
        to_np(start).astype(np.float64), 60, 20, serial=False, dictionary=True)
    e_img, e_obj = rel(to_np(delta), r_img), np.abs(obj / r_obj - 1).max()
    say("dictionary FISTA (node H, Eq. 5): image rel err %.3e, objective rel %.3e" % (e_img, e_obj))
    assert abs(L / r_L - 1) < 1e-10
    assert e_obj < 1e-10 and e_img < 1e-6


def test_fista_two_nodes_teacher_forced(tiny2):
    d, h = tiny2
    n = d["n_img"]
    rng = np.random.default_rng(32)
    model = to_dev(0.3 * d["truth"])
    rho = to_dev(0.002 * rng.standard_normal((n, n)))
    for p, own in ((0, "L"), (1, "H")):
        import torch
        local = torch.empty((n, n), device="cuda")
        h.major_cycle(p, model, local_out=local)
        psf = h.psf(p)
        start = to_dev(rng.standard_normal((n, n)))
        delta, obj, L, lam = h.minor_cycle_fista(p, local, start, rho_other=rho, n_iter=40,
                                                 power_iters=20, gamma_n=1.0, want_objective=True)
        r_img, r_obj, r_L, r_lam = _oracle_run(
            to_np(local).astype(np.float64), to_np(psf).astype(np.float64),
            to_np(rho).astype(np.float64), 1.0, h.info.ell_pix, h.info.delta_pix, own,
            to_np(start).astype(np.float64), 40, 20, serial=False)
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
        {k: to_np(to_dev(s)).astype(np.float64) for k, s in starts.items()}, n_iter=25,
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
