"""Serving loop on the GPU: every request's result is identical alone, in a
mix of concurrent requests, under a tight memory budget, and to the plain
one-call reconstruction; the footprint estimates bound what the handles
actually hold."""

import numpy as np
import pytest

from helpers import say

pytestmark = pytest.mark.gpu


def _serve():
    from paper_2507_22128_amd import serve
    return serve


@pytest.fixture(scope="module")
def requests_small():
    from paper_2507_22128_amd import synth
    say("case: 4 requests (48 antennas, 16 times, 128 / 256 images): msCLEAN and FISTA, "
        "1 and 2 partitions")
    d = synth.make_channels(n_chan=4, n_ant=48, n_time=16, sizes=(128, 256), seed=9)
    spec = [dict(method="msclean", n_partitions=2, n_cycles=3, niter=60, scales=(0, 2, 4)),
            dict(method="fista", n_partitions=1, n_cycles=2, fista_iter=15, power_iters=5),
            dict(method="msclean", n_partitions=1, n_cycles=2, niter=40, scales=(0, 3)),
            dict(method="fista", n_partitions=2, n_cycles=3, fista_iter=10, power_iters=4)]
    reqs = []
    for k, (c, s) in enumerate(zip(d["channels"], spec)):
        reqs.append(_serve().Request(uvw=d["uvw"], vis=c["vis"], freq_hz=c["freq_hz"],
                                     cell=c["cell"], n_pix=c["n_img"], flag=c["flag"],
                                     name="req%d" % k, power_seed=k, **s))
    return reqs


def _finals(results):
    return [r.final.cpu().numpy() for r in results]


def test_results_identical_alone_mixed_and_plain(requests_small):
    serve = _serve()
    reqs = requests_small
    alone = []
    with serve.Server(hbm_budget=64 << 30, workers=1) as srv:
        for r in reqs:
            alone.append(srv.submit(r).result(timeout=300))
    with serve.Server(hbm_budget=64 << 30, workers=3) as srv:
        futs = [srv.submit(r) for r in reqs]
        mixed = [f.result(timeout=300) for f in futs]
    say("mixed: max concurrent cycles %d, max resident requests %d"
        % (srv.max_concurrent_cycles, srv.max_resident_jobs))
    plain = [f.cpu().numpy() for f, _ in serve.run_serial(reqs)]
    for r, a, m, p in zip(reqs, _finals(alone), _finals(mixed), plain):
        assert np.array_equal(a, m), "%s differs alone vs mixed" % r.name
        assert np.array_equal(a, p), "%s differs from the one-call reconstruction" % r.name
        assert np.abs(a).max() > 0
    for res in alone + mixed:
        assert res.device_bytes <= res.footprint[0], res.name
        assert res.device_peak_bytes <= res.footprint[1], res.name
        assert res.latency > 0 and res.n_valid > 0


def test_tight_budget_admits_in_turn(requests_small):
    serve = _serve()
    reqs = requests_small
    ex = serve.ImagerExecutor()
    peaks = [ex.footprint(r)[1] for r in reqs]
    budget = int(1.02 * max(peaks))
    with serve.Server(hbm_budget=budget, workers=3) as srv:
        futs = [srv.submit(r) for r in reqs]
        res = [f.result(timeout=300) for f in futs]
    say("tight budget %d: max reserved %d, admission waits %d"
        % (budget, srv.max_reserved, srv.admission_waits))
    assert srv.max_reserved <= budget
    assert srv.admission_waits >= 1
    with serve.Server(hbm_budget=64 << 30, workers=1) as srv:
        ref = [srv.submit(r).result(timeout=300) for r in reqs]
    for a, b in zip(_finals(res), _finals(ref)):
        assert np.array_equal(a, b)
    from paper_2507_22128_amd import imager
    with serve.Server(hbm_budget=min(peaks) // 2, workers=1) as srv:
        with pytest.raises(imager.ImagerError) as e:
            srv.submit(reqs[0]).result(timeout=60)
    assert e.value.code == imager.ENOMEM
