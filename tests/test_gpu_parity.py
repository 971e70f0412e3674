"""Parity of the HIP library with the FP64 oracle (GPU required).

Every comparison uses the same seeded inputs on both sides: the oracle
consumes the exact arrays handed to the library (complex64 visibilities are
up-cast exactly).  Floating-point results must agree to a relative L2 error
of 1e-5; integer decisions (weights' cells, partition membership, ell) must
agree bit for bit.
"""

import numpy as np
import pytest

from helpers import (decentral, geometry, imaging, oracle_weights, random_model, rel, say,
                     to_dev, to_np, uv, workload)

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _imager():
    from paper_2507_22128_amd import imager
    return imager


@pytest.fixture(scope="module")
def tiny():
    say("case: tiny workload, 1 partition, uniform weights")
    d = workload("tiny")
    h = _imager().Imager.create(d, n_partitions=1, weighting="uniform")
    yield d, h
    h.destroy()


def test_tiny_weights_and_members_bitwise(tiny):
    d, h = tiny
    n = d["n_img"]
    w = oracle_weights(d, n)
    assert np.array_equal(h.vis_index(0), np.arange(len(w)))
    assert np.array_equal(h.vis_weight(0), w.astype(np.float32))
    assert h.sum_w(0) == pytest.approx(w.sum(), rel=1e-13)


def test_tiny_dirty_image(tiny):
    import torch
    d, h = tiny
    n = d["n_img"]
    u, v = uv(d)
    w = oracle_weights(d, n)
    ref = imaging.dirty_image(u, v, d["vis"], w, n, d["cell"])
    got = to_np(h.major_cycle(0, torch.zeros((n, n), device="cuda")))
    say("tiny dirty rel err %.3e" % rel(got, ref))
    assert rel(got, ref) < TOL
    vis = to_dev(d["vis"], "complex64")
    got2 = to_np(h.grid(0, vis))
    assert rel(got2, ref) < TOL


def test_tiny_degrid(tiny):
    d, h = tiny
    n = d["n_img"]
    u, v = uv(d)
    model = random_model(n, np.random.default_rng(1))
    ref = imaging.Operator(u, v, d["cell"], n).forward(model)
    got = to_np(h.degrid(0, to_dev(model)))
    say("tiny degrid rel err %.3e" % rel(got, ref))
    assert rel(got, ref) < TOL


def test_tiny_grid_adjoint(tiny):
    d, h = tiny
    n = d["n_img"]
    u, v = uv(d)
    w = oracle_weights(d, n)
    rng = np.random.default_rng(2)
    y = (rng.standard_normal(len(u)) + 1j * rng.standard_normal(len(u))).astype(np.complex64)
    ref = imaging.Operator(u, v, d["cell"], n).adjoint(w * y.astype(np.complex128)).real
    got = to_np(h.grid(0, to_dev(y, "complex64"), mode=_imager().GRID_UNNORMALIZED))
    say("tiny grid rel err %.3e" % rel(got, ref))
    assert rel(got, ref) < TOL


def test_tiny_psf(tiny):
    d, h = tiny
    n = d["n_img"]
    u, v = uv(d)
    w = oracle_weights(d, n)
    ref = imaging.psf2(u, v, w, n, d["cell"])
    got = to_np(h.psf(0))
    say("tiny psf rel err %.3e" % rel(got, ref))
    assert rel(got, ref) < TOL
    assert np.unravel_index(np.argmax(got), got.shape) == (n, n)
    assert abs(got[n, n] - 1.0) < 1e-5


def test_tiny_major_cycle_repeatable(tiny):
    import torch
    d, h = tiny
    n = d["n_img"]
    u, v = uv(d)
    w = oracle_weights(d, n)
    model = 0.5 * d["truth"]
    ref, _ = imaging.residual_image(u, v, d["vis"], w, model, d["cell"])
    m = to_dev(model)
    a = h.major_cycle(0, m)
    b = h.major_cycle(0, m)
    say("tiny major cycle rel err %.3e" % rel(to_np(a), ref))
    assert rel(to_np(a), ref) < TOL
    # no atomics anywhere and a fixed flush order: bit for bit the same
    assert torch.equal(a, b), "two identical major cycles differ"


# block side (tile), support, chunk cap, flag rate, weighting: every (W, blk)
# family of kernels, chunks far below and far above the block occupancy
VARIANTS = [
    dict(tile=8, support=6, chunk=64, flag_rate=0.1, weighting="natural"),
    dict(tile=4, support=12, chunk=100000, flag_rate=0.0, weighting="uniform"),
    dict(tile=8, support=4, chunk=777, flag_rate=0.3, weighting="uniform"),
    dict(tile=4, support=10, chunk=4096, flag_rate=0.02, weighting="natural"),
    dict(tile=4, support=8, chunk=16, flag_rate=0.05, weighting="uniform"),
    dict(tile=4, support=6, chunk=33, flag_rate=0.0, weighting="natural"),
    dict(tile=4, support=4, chunk=1000, flag_rate=0.5, weighting="uniform"),
]


@pytest.mark.parametrize("var", VARIANTS, ids=lambda v: "T%d-W%d-C%d" % (v["tile"], v["support"], v["chunk"]))
def test_variants_dirty_and_residual(var):
    say("case: variant %s" % var)
    d = workload("tiny", n_time=20)
    n = d["n_img"]
    rng = np.random.default_rng(var["chunk"])
    flag = (rng.random(len(d["vis"])) < var["flag_rate"]).astype(np.uint8)
    valid = flag == 0
    h = _imager().Imager.create(d, n_partitions=1, weighting=var["weighting"], tile=var["tile"],
                                support=var["support"], chunk=var["chunk"], flag=flag)
    try:
        u, v = uv(d)
        w = oracle_weights(d, n, valid=valid, uniform=var["weighting"] == "uniform")
        assert np.array_equal(h.vis_index(0), np.nonzero(valid)[0])
        assert np.array_equal(h.vis_weight(0), w[valid].astype(np.float32))
        model = random_model(n, rng)
        sel = valid
        ref, _ = imaging.residual_image(u[sel], v[sel], d["vis"][sel], w[sel], model, d["cell"],
                                        support=var["support"])
        got = to_np(h.major_cycle(0, to_dev(model)))
        say("variant residual rel err %.3e" % rel(got, ref))
        assert rel(got, ref) < TOL
    finally:
        h.destroy()


# ------------------------------------------------------------------ two partitions

@pytest.fixture(scope="module")
def medium():
    say("case: decentral workload (16 time steps), 2 partitions")
    d = workload("decentral", n_time=16)
    h = _imager().Imager.create(d, n_partitions=2, weighting="uniform")
    yield d, h
    h.destroy()


def _medium_oracle(d):
    n = d["n_img"]
    u, v = uv(d)
    w = oracle_weights(d, n)
    low, high, ell = imaging.partition(u, v, n, d["cell"])
    return u, v, w, low, high, ell


def test_partition_bitwise(medium):
    d, h = medium
    u, v, w, low, high, ell = _medium_oracle(d)
    assert h.info.ell_pix == ell
    assert np.array_equal(h.vis_index(0), np.nonzero(low)[0])
    assert np.array_equal(h.vis_index(1), np.nonzero(high)[0])
    for p, mask in ((0, low), (1, high)):
        assert np.array_equal(h.vis_weight(p), w[mask].astype(np.float32))
        assert h.sum_w(p) == pytest.approx(w[mask].sum(), rel=1e-12)


def test_partition_residuals_psfs_and_composition(medium):
    d, h = medium
    n = d["n_img"]
    u, v, w, low, high, ell = _medium_oracle(d)
    rng = np.random.default_rng(5)
    model = random_model(n, rng)
    rho = 0.01 * random_model(n, rng)
    psfs, locals_ = {}, {}
    for p, mask in ((0, low), (1, high)):
        psfs[p] = imaging.psf2(u[mask], v[mask], w[mask], n, d["cell"])
        got_psf = to_np(h.psf(p))
        say("part %d psf rel err %.3e" % (p, rel(got_psf, psfs[p])))
        assert rel(got_psf, psfs[p]) < TOL
        locals_[p], _ = imaging.residual_image(u[mask], v[mask], d["vis"][mask], w[mask], model,
                                               d["cell"])
    wl, wh = w[low].sum(), w[high].sum()
    import torch
    for p, own in ((0, "L"), (1, "H")):
        gamma, mu = decentral.weights_schedule(2, (wl, wh)[p], (wh, wl)[p])
        local = torch.empty((n, n), device="cuda")
        out = h.major_cycle(p, to_dev(model), to_dev(rho), gamma, mu, local_out=local)
        say("part %d local residual rel err %.3e" % (p, rel(to_np(local), locals_[p])))
        assert rel(to_np(local), locals_[p]) < TOL
        ref = decentral.compose_dirty(locals_[p], rho, psfs[1 - p], ell, 1.0, own, gamma, mu)
        say("part %d composed residual rel err %.3e" % (p, rel(to_np(out), ref)))
        assert rel(to_np(out), ref) < TOL
        ref_psf = decentral.compose_psf(psfs[p], psfs[1 - p], ell, 1.0, own, gamma, mu)
        got_psf = to_np(h.composed_psf(p, gamma, mu))
        say("part %d composed psf rel err %.3e" % (p, rel(got_psf, ref_psf)))
        assert rel(got_psf, ref_psf) < TOL
    # first cycle: gamma = 1, mu = 0, no rho
    out1 = to_np(h.major_cycle(0, to_dev(model)))
    ref1 = decentral.compose_dirty(locals_[0], None, None, ell, 1.0, "L", 1.0, 0.0)
    assert rel(out1, ref1) < TOL


def test_concurrent_nodes_equal_single_calls(medium):
    """Both nodes' cycles on their own streams give each node's result bit
    for bit, and twice in a row (work buffers are per node)."""
    import torch
    d, h = medium
    n = d["n_img"]
    rng = np.random.default_rng(9)
    models = [to_dev(random_model(n, rng)) for _ in range(2)]
    rhos = [to_dev(0.01 * random_model(n, rng)) for _ in range(2)]
    gam, mus = [0.6, 0.4], [0.4, 0.6]
    single = [h.major_cycle(p, models[p], rhos[p], gam[p], mus[p]) for p in (0, 1)]
    for _ in range(2):
        both = h.major_cycle_nodes(models, rhos, gam, mus)
        for p in (0, 1):
            assert torch.equal(both[p], single[p]), "node %d differs" % p
    # one node with the PSF term of Eq. 7, the other without
    mus = [0.0, 0.6]
    single = [h.major_cycle(p, models[p], rhos[p], gam[p], mus[p]) for p in (0, 1)]
    both = h.major_cycle_nodes(models, rhos, gam, mus)
    for p in (0, 1):
        assert torch.equal(both[p], single[p]), "node %d differs (mu = %g)" % (p, mus[p])
    # two calls in a row with different rho, no synchronisation between them:
    # each call's PSF term reads its own rho (the terms' work buffers are reused)
    mus = [0.4, 0.6]
    rhos_b = [to_dev(0.02 * random_model(n, rng)) for _ in range(2)]
    single_a = [h.major_cycle(p, models[p], rhos[p], gam[p], mus[p]) for p in (0, 1)]
    single_b = [h.major_cycle(p, models[p], rhos_b[p], gam[p], mus[p]) for p in (0, 1)]
    out_a = h.major_cycle_nodes(models, rhos, gam, mus)
    out_b = h.major_cycle_nodes(models, rhos_b, gam, mus)
    for p in (0, 1):
        assert torch.equal(out_a[p], single_a[p]), "first of two calls, node %d" % p
        assert torch.equal(out_b[p], single_b[p]), "second of two calls, node %d" % p


def test_composite_degrid(medium):
    d, h = medium
    n = d["n_img"]
    u, v, w, low, high, ell = _medium_oracle(d)
    rng = np.random.default_rng(6)
    model = random_model(n, rng)
    rho = 0.05 * random_model(n, rng)
    import torch
    local = torch.empty((n, n), device="cuda")
    h.major_cycle(1, to_dev(model), to_dev(rho), 0.5, 0.0, composite=True, local_out=local)
    ref, _ = imaging.residual_image(u[high], v[high], d["vis"][high], w[high], model + rho,
                                    d["cell"])
    assert rel(to_np(local), ref) < TOL


def test_exchange_and_final_combination(medium):
    d, h = medium
    n = d["n_img"]
    _, _, _, _, _, ell = _medium_oracle(d)
    rng = np.random.default_rng(7)
    a, b = rng.standard_normal((2, n, n)).astype(np.float32)
    ra, rb = rng.standard_normal((2, n, n)).astype(np.float32)
    ta, tb = to_dev(ra), to_dev(rb)
    h.exchange(to_dev(a), to_dev(b), ta, tb)
    a64, b64 = a.astype(np.float64), b.astype(np.float64)
    # node L's aggregate: rho_H + Phi_H - Gamma_H ibar_L with Phi_H = Gamma_H ibar_H
    ref_a = decentral.update_rho(ra.astype(np.float64), decentral.exchange(b64, ell, 1.0, "H"),
                                 a64, ell, 1.0, "L")
    ref_b = decentral.update_rho(rb.astype(np.float64), decentral.exchange(a64, ell, 1.0, "L"),
                                 b64, ell, 1.0, "H")
    assert rel(to_np(ta) - ra, ref_a - ra) < TOL
    assert rel(to_np(tb) - rb, ref_b - rb) < TOL
    fin = to_np(h.combine_final(to_dev(a), to_dev(b)))
    assert np.array_equal(fin, decentral.combine([a64, b64]))


def test_errors_are_reported(medium):
    import torch
    d, h = medium
    imager = _imager()
    with pytest.raises(imager.ImagerError) as e:
        h.minor_cycle_msclean(0, torch.zeros((d["n_img"],) * 2, device="cuda"),
                              torch.zeros((2 * d["n_img"],) * 2, device="cuda"), [0, 4], gain=2.0)
    assert e.value.code == imager.EINVAL
    with pytest.raises(imager.ImagerError):
        h.major_cycle(5, torch.zeros((d["n_img"],) * 2, device="cuda"))
    # an empty partition is refused at create
    with pytest.raises(imager.ImagerError) as e:
        imager.Imager.create(d, n_partitions=2, ell=1e9)
    assert e.value.code == imager.EINVAL
    # hbm budget far below the footprint
    with pytest.raises(imager.ImagerError) as e:
        imager.Imager.create(d, n_partitions=2, hbm_budget=1 << 20)
    assert e.value.code == imager.ENOMEM


def test_all_flagged_is_refused():
    d = workload("tiny", n_time=4)
    imager = _imager()
    with pytest.raises(imager.ImagerError) as e:
        imager.Imager.create(d, n_partitions=1, flag=np.ones(len(d["vis"]), np.uint8))
    assert e.value.code == imager.EINVAL


@pytest.mark.parametrize("n_pix", [64, 2048])
def test_smallest_and_largest_image_sizes(n_pix):
    """N = 64 and N = 2048 (grids of 128 and 4096, PSF grids of 256 and 8192:
    the smallest and largest transform lengths the library builds), against
    the direct Fourier sums at sampled pixels."""
    from oracle import dft
    say("case: tiny array (10 time steps), N = %d" % n_pix)
    d = workload("tiny", n_time=10)
    h = _imager().Imager.create(d, n_pix=n_pix, n_partitions=1, weighting="uniform")
    try:
        n = n_pix
        u, v = uv(d)
        w = imaging.uniform_weights(u, v, n, d["cell"])
        rng = np.random.default_rng(n)
        iy = np.concatenate([[n // 2], rng.integers(0, n, 12)])
        ix = np.concatenate([[n // 2], rng.integers(0, n, 12)])
        q = (n // 2 + 5, n // 2 - 3)
        model = np.zeros((n, n))
        model[q] = 0.5
        pred = dft.forward_points([0.5], [q[0]], [q[1]], u, v, d["cell"], n)
        r = w * (d["vis"] - pred)
        ref = dft.adjoint_at(r, u, v, d["cell"], n, iy, ix).real / w.sum()
        got = to_np(h.major_cycle(0, to_dev(model)))[iy, ix].astype(np.float64)
        err = np.abs(got - ref).max() / np.abs(ref).max()
        dy, dx = rng.integers(-8, 9, 10), rng.integers(-8, 9, 10)
        pref = dft.adjoint_at(w, u, v, d["cell"], 2 * n, n + dy, n + dx).real / w.sum()
        pgot = to_np(h.psf(0))[n + dy, n + dx].astype(np.float64)
        perr = np.abs(pgot - pref).max() / np.abs(pref).max()
        say("N = %d: residual max err %.3e, PSF max err %.3e" % (n, err, perr))
        assert err < TOL and perr < TOL
    finally:
        h.destroy()


@pytest.mark.parametrize("n_pix", [64, 128])
def test_two_partitions_small_images(n_pix):
    """The two-node cycle at the smallest image sizes (Gamma filters of 64 and
    128 points, PSF convolutions of 128 and 256): each node's composed
    residual (Eq. 7) against the oracle, and equal bit for bit to the
    single-node call."""
    import torch
    say("case: tiny array (10 time steps), N = %d, 2 partitions" % n_pix)
    d = workload("tiny", n_time=10)
    n = n_pix
    h = _imager().Imager.create(d, n_pix=n, n_partitions=2, weighting="uniform")
    try:
        u, v = uv(d)
        w = imaging.uniform_weights(u, v, n, d["cell"])
        low, high, ell = imaging.partition(u, v, n, d["cell"])
        assert h.info.ell_pix == ell
        rng = np.random.default_rng(n + 1)
        model = random_model(n, rng, n_points=6)
        rho = 0.01 * random_model(n, rng, n_points=6)
        psfs, locals_ = {}, {}
        for p, mask in ((0, low), (1, high)):
            psfs[p] = imaging.psf2(u[mask], v[mask], w[mask], n, d["cell"])
            locals_[p], _ = imaging.residual_image(u[mask], v[mask], d["vis"][mask], w[mask],
                                                   model, d["cell"])
        wl, wh = w[low].sum(), w[high].sum()
        gm, mus = [], []
        for p in (0, 1):
            g, m = decentral.weights_schedule(2, (wl, wh)[p], (wh, wl)[p])
            gm.append(g)
            mus.append(m)
        models = [to_dev(model), to_dev(model)]
        rhos = [to_dev(rho), to_dev(rho)]
        both = h.major_cycle_nodes(models, rhos, gm, mus)
        for p, own in ((0, "L"), (1, "H")):
            ref = decentral.compose_dirty(locals_[p], rho, psfs[1 - p], ell, 1.0, own, gm[p],
                                          mus[p])
            err = rel(to_np(both[p]), ref)
            say("N = %d part %d composed residual rel err %.3e" % (n, p, err))
            assert err < TOL
            single = h.major_cycle(p, models[p], rhos[p], gm[p], mus[p])
            assert torch.equal(both[p], single), "node %d differs from its single call" % p
    finally:
        h.destroy()


def test_windows_wrapping_the_grid_edge():
    """A cell size that puts the outermost visibilities within half a support
    of the grid's edge: their footprints wrap around (the oracle's gridding
    takes cell indices modulo Ng), and the transforms and flush must cover the
    whole grid instead of the box of the chunk windows."""
    say("case: tiny array (6 time steps), N = 64, cell 0.499 / max |u|: footprints wrap")
    d = workload("tiny", n_time=6)
    u, v = uv(d)
    cell = 0.499 / max(np.abs(u).max(), np.abs(v).max())
    n = 64
    h = _imager().Imager.create(uvw=d["uvw"], vis=d["vis"], freq_hz=d["freq_hz"], cell=cell,
                                n_pix=n, n_partitions=1, weighting="uniform")
    try:
        w = imaging.uniform_weights(u, v, n, cell)
        model = random_model(n, np.random.default_rng(41), n_points=8)
        ref, _ = imaging.residual_image(u, v, d["vis"], w, model, cell)
        got = to_np(h.major_cycle(0, to_dev(model)))
        err = rel(got, ref)
        g = geometry.grid_coord(u, 2 * n, cell)
        say("max |grid coordinate - Ng/2| = %.2f of %d: residual rel err %.3e"
            % (np.abs(g - n).max(), n, err))
        assert np.abs(g - n).max() > n - 4  # some footprints cross the edge
        assert err < TOL
    finally:
        h.destroy()
