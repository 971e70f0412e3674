"""Batched channels and the work-layout autotuner (GPU required).

The fused batch runs the same per-chunk and per-cell device code as a
single handle, so its residuals must equal each member's own
imager_major_cycle bit for bit, in eager, graph and per-channel-loop modes,
and after re-chunking.  Two members are also checked against the FP64
oracle at the usual 1e-5 relative L2 bound.
"""

import numpy as np
import pytest

from helpers import imaging, geometry, random_model, rel, say, to_dev, to_np

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _imager():
    from paper_2507_22128_amd import imager
    return imager


def _channels():
    from paper_2507_22128_amd import synth
    return synth.make_channels(n_chan=5, n_ant=48, n_time=16, sizes=(64, 128, 256), seed=7)


def _create(d, c, **kw):
    return _imager().Imager.create(uvw=d["uvw"], vis=c["vis"], freq_hz=c["freq_hz"],
                                   cell=c["cell"], n_pix=c["n_img"], flag=c["flag"],
                                   n_partitions=1, weighting="uniform", **kw)


@pytest.fixture(scope="module")
def chans():
    say("case: 5 channels (48 antennas, 16 times), sizes 64/128/256, flags 0-60 %")
    d = _channels()
    members = [_create(d, c, chunk=256) for c in d["channels"]]
    rng = np.random.default_rng(21)
    models = [to_dev(random_model(c["n_img"], rng, n_points=12)) for c in d["channels"]]
    yield d, members, models
    for m in members:
        m.destroy()


def _singles(members, models):
    return [to_np(m.major_cycle(0, x)) for m, x in zip(members, models)]


def test_batch_equals_single_handles_bitwise(chans):
    d, members, models = chans
    ref = _singles(members, models)
    b = _imager().Batch(members)
    try:
        info = b.info()
        assert info.n_members == len(members)
        assert info.n_vis == sum(m.n_vis(0) for m in members)
        assert info.n_chunks == sum(m.info.n_chunks[0] for m in members)
        assert info.n_sets == 1  # small grids: one fused launch
        for mode in (dict(), dict(loop=True), dict(graph=True)):
            got = [to_np(r) for r in b.major_cycle(models, **mode)]
            say("batch mode %s: max |diff| %.3e" % (mode, max(np.abs(g - r).max()
                                                                for g, r in zip(got, ref))))
            for g, r in zip(got, ref):
                assert np.array_equal(g, r)
    finally:
        b.destroy()


def test_batch_graph_replays_match_eager(chans):
    """Replays of one captured graph with eager work and new model values in
    between: every replay equals the eager batch for the current models."""
    import torch
    d, members, models = chans
    b = _imager().Batch(members)
    try:
        mods = [x.clone() for x in models]
        res = [torch.empty_like(x) for x in models]
        for rep in range(4):
            b.major_cycle(mods, res, graph=True)
            assert b.info().graph_ready == 1
            got = [to_np(r) for r in res]
            eager = [to_np(r) for r in b.major_cycle(mods)]
            for g, e in zip(got, eager):
                assert np.array_equal(g, e), "replay %d differs from eager" % rep
            # eager work between replays, then new values in the same buffers
            members[0].major_cycle(0, mods[0])
            torch.cuda.synchronize()
            for x in mods:
                x.mul_(0.5).add_(0.01)
        # new residual pointers: a new capture, same results
        res2 = [torch.empty_like(x) for x in models]
        b.major_cycle(mods, res2, graph=True)
        eager = [to_np(r) for r in b.major_cycle(mods)]
        for g, e in zip(res2, eager):
            assert np.array_equal(to_np(g), e)
    finally:
        b.destroy()


def test_batch_members_against_oracle(chans):
    d, members, models = chans
    b = _imager().Batch(members)
    try:
        got = [to_np(r) for r in b.major_cycle(models, graph=True)]
    finally:
        b.destroy()
    for k in (0, 3):
        c = d["channels"][k]
        n = c["n_img"]
        u, v = geometry.uv_lambda(d["uvw"], c["freq_hz"])
        valid = c["flag"] == 0
        w = imaging.uniform_weights(u, v, n, c["cell"], valid=valid)
        ref, _ = imaging.residual_image(u[valid], v[valid], c["vis"][valid], w[valid],
                                        to_np(models[k]).astype(np.float64), c["cell"])
        err = rel(got[k], ref)
        say("channel %d (N=%d, %.0f%% flagged): rel err %.3e" % (k, n, 100 * c["flag_frac"], err))
        assert err < TOL


def test_batch_member_sets_bitwise():
    """With a cache budget, members whose grids and chunk windows together
    exceed it run in several consecutive sets; every mode, with sets and
    with the default single set, still equals each member's own cycle bit
    for bit."""
    from paper_2507_22128_amd import synth
    say("case: 3 channels of N = 2048 (4096^2 grids of 134 MB each), sets of 128 MB and one set")
    d = synth.make_channels(n_chan=3, n_ant=24, n_time=8, sizes=(2048,), seed=9)
    members = [_create(d, c, chunk=256) for c in d["channels"]]
    try:
        rng = np.random.default_rng(22)
        models = [to_dev(random_model(c["n_img"], rng, n_points=12, smooth=False))
                  for c in d["channels"]]
        ref = _singles(members, models)
        b = _imager().Batch(members)
        try:
            b.set_bytes(128 << 20)  # half of the last-level cache: one set per member
            assert b.info().n_sets == 3
            for mode in (dict(), dict(graph=True)):
                got = [to_np(r) for r in b.major_cycle(models, **mode)]
                for g, r in zip(got, ref):
                    assert np.array_equal(g, r)
            # the default: one fused launch for all
            b.set_bytes(0)
            assert b.info().n_sets == 1
            for mode in (dict(), dict(graph=True)):
                got = [to_np(r) for r in b.major_cycle(models, **mode)]
                for g, r in zip(got, ref):
                    assert np.array_equal(g, r)
        finally:
            b.destroy()
    finally:
        for m in members:
            m.destroy()


def test_set_chunk_equals_fresh_create(chans):
    d, members, models = chans
    c = d["channels"][1]
    h = _create(d, c, chunk=256)
    try:
        h.set_chunk(48)
        assert h.info.chunk == 48
        fresh = _create(d, c, chunk=48)
        try:
            assert fresh.info.n_chunks[0] == h.info.n_chunks[0]
            a = to_np(h.major_cycle(0, models[1]))
            f = to_np(fresh.major_cycle(0, models[1]))
            assert np.array_equal(a, f)
        finally:
            fresh.destroy()
    finally:
        h.destroy()


def test_batch_autotune_keeps_results(chans):
    d, members, models = chans
    hs = [_create(d, c, chunk=256) for c in d["channels"]]
    b = _imager().Batch(hs)
    try:
        caps = (32, 128, 512)
        chosen, times = b.autotune(caps, reps=2)
        say("batch autotune: chosen %d, times %s" % (chosen, times))
        assert chosen in caps and set(times) == set(caps)
        assert times[chosen] == min(times.values())
        assert all(h.info.chunk == chosen for h in hs)
        assert b.info().chunk == chosen
        ref = [to_np(h.major_cycle(0, x)) for h, x in zip(hs, models)]
        got = [to_np(r) for r in b.major_cycle(models, graph=True)]
        for g, r in zip(got, ref):
            assert np.array_equal(g, r)
        # the same chunk cap at create gives the same tables, hence the same bits
        fresh = _create(d, d["channels"][2], chunk=chosen)
        try:
            assert np.array_equal(to_np(fresh.major_cycle(0, models[2])), ref[2])
        finally:
            fresh.destroy()
    finally:
        b.destroy()
        for h in hs:
            h.destroy()


def test_create_time_autotuner_and_support_rule(chans):
    d, members, models = chans
    c = d["channels"][0]
    h = _create(d, c, support=0, tolerance=1e-5, autotune=True)
    try:
        assert h.info.support == 8
        log = h.tune_log()
        say("create autotune log %s -> tile %d chunk %d" % (log, h.info.tile, h.info.chunk))
        assert {t for t, _, _ in log} == {4, 8}
        assert {k for _, k, _ in log} == {256, 512, 1024, 2048, 4096}
        best = min(log, key=lambda e: e[2])
        assert (h.info.tile, h.info.chunk) == best[:2]
        # the tuned handle is the same operator: oracle parity
        n = c["n_img"]
        u, v = geometry.uv_lambda(d["uvw"], c["freq_hz"])
        valid = c["flag"] == 0
        w = imaging.uniform_weights(u, v, n, c["cell"], valid=valid)
        ref, _ = imaging.residual_image(u[valid], v[valid], c["vis"][valid], w[valid],
                                        to_np(models[0]).astype(np.float64), c["cell"])
        assert rel(to_np(h.major_cycle(0, models[0])), ref) < TOL
    finally:
        h.destroy()
    h6 = _create(d, c, support=0, tolerance=1e-3, tile=8, chunk=512, autotune=True)
    try:
        assert h6.info.support == 6 and h6.info.tile == 8 and h6.info.chunk == 512
        assert h6.tune_log() == []  # nothing left to tune
    finally:
        h6.destroy()
    with pytest.raises(_imager().ImagerError) as e:
        _create(d, c, support=0, tolerance=1e-12)
    assert e.value.code == _imager().EINVAL


def test_batch_rejects_mismatched_members(chans):
    d, members, models = chans
    im = _imager()
    other = _create(d, d["channels"][0], support=6, tile=8)
    try:
        with pytest.raises(im.ImagerError) as e:
            im.Batch([members[0], other])
        assert e.value.code == im.EINVAL
        with pytest.raises(im.ImagerError):
            im.Batch([members[0], members[0]])
    finally:
        other.destroy()


def test_batch_nine_channels_against_oracle():
    """Nine channels with uneven observation lengths (T_c uniform in 6 .. 12
    time steps) and flags, images 128 - 512 plus one of 2048^2: every
    member's residual from the fused batch (graph replay) against the FP64
    oracle."""
    from paper_2507_22128_amd import synth
    say("case: 8 channels (40 antennas, T_c in 6..12, sizes 128/256/512) + 1 channel at 2048^2")
    sets = [synth.make_channels(n_chan=8, n_ant=40, n_time=12, t_min=6, sizes=(128, 256, 512),
                                seed=31),
            synth.make_channels(n_chan=1, n_ant=40, n_time=12, t_min=6, sizes=(2048,), seed=32,
                                f_lo=1.4e9, f_hi=1.4e9)]
    pairs = [(d, c) for d in sets for c in d["channels"]]
    assert len(pairs) == 9 and any(c["n_img"] == 2048 for _, c in pairs)
    assert len({c["n_time"] for _, c in pairs}) > 1
    members = [_create(d, c, chunk=256) for d, c in pairs]
    rng = np.random.default_rng(23)
    models = [to_dev(random_model(c["n_img"], rng, n_points=10, smooth=False)) for _, c in pairs]
    b = _imager().Batch(members)
    try:
        got = [to_np(r) for r in b.major_cycle(models, graph=True)]
        again = [to_np(r) for r in b.major_cycle(models, graph=True)]
    finally:
        b.destroy()
        for m in members:
            m.destroy()
    for k, ((d, c), g) in enumerate(zip(pairs, got)):
        assert np.array_equal(g, again[k])
        n = c["n_img"]
        u, v = geometry.uv_lambda(d["uvw"], c["freq_hz"])
        valid = c["flag"] == 0
        w = imaging.uniform_weights(u, v, n, c["cell"], valid=valid)
        ref, _ = imaging.residual_image(u[valid], v[valid], c["vis"][valid], w[valid],
                                        to_np(models[k]).astype(np.float64), c["cell"])
        err = rel(g, ref)
        say("channel %d (N=%d, T_c=%d, %d unflagged): rel err %.3e"
            % (k, n, c["n_time"], int(valid.sum()), err))
        assert err < TOL
