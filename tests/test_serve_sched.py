"""Scheduling logic of the serving loop on the CPU (a fake executor stands
in for the GPU): FIFO admission by memory footprint, the budget is never
exceeded, requests that can never fit are refused, resident requests are
advanced one cycle at a time and interleave, failures are contained."""

import threading
import time

import pytest

from paper_2507_22128_amd import imager, serve


class Req:
    def __init__(self, name, peak, resident, cycles, cycle_s=0.002, fail_at=None):
        self.name, self.peak, self.resident, self.n_cycles = name, peak, resident, cycles
        self.cycle_s, self.fail_at = cycle_s, fail_at


class FakeExecutor:
    def __init__(self):
        self.lock = threading.Lock()
        self.log = []          # (event, name, cycle)
        self.live = 0
        self.max_live = 0

    def footprint(self, req):
        return req.resident, req.peak

    def start(self, req):
        with self.lock:
            self.log.append(("start", req.name, 0))
        time.sleep(0.001)
        return dict(req=req, acc=0)

    def cycle(self, st, k):
        req = st["req"]
        with self.lock:
            self.live += 1
            self.max_live = max(self.max_live, self.live)
            self.log.append(("cycle", req.name, k))
        time.sleep(req.cycle_s)
        with self.lock:
            self.live -= 1
        if req.fail_at == k:
            raise RuntimeError("cycle %d of %s failed" % (k, req.name))
        st["acc"] = st["acc"] * 31 + k

    def finish(self, st):
        return dict(final=st["acc"], models=[], n_valid=1, device_bytes=st["req"].resident,
                    device_peak_bytes=st["req"].peak)

    def measured_bytes(self, st):
        return st["req"].resident

    def release(self, st):
        with self.lock:
            self.log.append(("release", st["req"].name, 0))


def test_admission_respects_budget_and_fifo():
    ex = FakeExecutor()
    reqs = [Req("r%d" % i, peak=40, resident=30, cycles=3) for i in range(6)]
    with serve.Server(hbm_budget=100, workers=3, executor=ex) as srv:
        futs = [srv.submit(r) for r in reqs]
        res = [f.result(timeout=30) for f in futs]
    assert srv.max_reserved <= 100
    # peaks of 40 while building, 30 resident: at most 3 resident at once
    assert srv.max_resident_jobs <= 3
    assert srv.admit_order == [r.name for r in reqs]
    assert [r.final for r in res] == [((0 * 31 + 1) * 31 + 2) * 31 + 3] * 6
    assert all(r.n_cycles == 3 and r.finished >= r.admitted >= r.arrival for r in res)


def test_request_larger_than_budget_is_refused():
    ex = FakeExecutor()
    with serve.Server(hbm_budget=50, workers=2, executor=ex) as srv:
        big = srv.submit(Req("big", peak=60, resident=10, cycles=1))
        ok = srv.submit(Req("ok", peak=50, resident=10, cycles=1))
        with pytest.raises(imager.ImagerError) as e:
            big.result(timeout=10)
        assert e.value.code == imager.ENOMEM
        assert ok.result(timeout=10).name == "ok"


def test_one_at_a_time_when_two_do_not_fit():
    ex = FakeExecutor()
    with serve.Server(hbm_budget=100, workers=4, executor=ex) as srv:
        futs = [srv.submit(Req("r%d" % i, peak=60, resident=60, cycles=2)) for i in range(3)]
        [f.result(timeout=30) for f in futs]
    assert srv.max_resident_jobs == 1 and srv.max_reserved <= 100
    assert srv.admission_waits >= 1
    # each request's cycles complete before the next one starts
    order = [(e, n) for e, n, _ in ex.log if e in ("start", "release")]
    assert order == [("start", "r0"), ("release", "r0"), ("start", "r1"), ("release", "r1"),
                     ("start", "r2"), ("release", "r2")]


def test_continuous_batching_interleaves_cycles():
    """A short request that arrives while a long one runs joins at a cycle
    boundary and finishes first; with one worker the cycles alternate."""
    ex = FakeExecutor()
    with serve.Server(hbm_budget=1000, workers=1, executor=ex) as srv:
        long = srv.submit(Req("long", peak=10, resident=10, cycles=8, cycle_s=0.01))
        time.sleep(0.03)
        short = srv.submit(Req("short", peak=10, resident=10, cycles=2, cycle_s=0.01))
        rs, rl = short.result(timeout=30), long.result(timeout=30)
    assert rs.finished < rl.finished
    cyc = [n for e, n, _ in ex.log if e == "cycle"]
    first_short = cyc.index("short")
    assert "long" in cyc[first_short + 1:]  # the long one was not run to the end first
    assert [k for e, n, k in ex.log if e == "cycle" and n == "long"] == list(range(1, 9))


def test_concurrent_workers_and_failure_containment():
    ex = FakeExecutor()
    with serve.Server(hbm_budget=1000, workers=4, executor=ex) as srv:
        futs = [srv.submit(Req("r%d" % i, peak=10, resident=10, cycles=4, cycle_s=0.01,
                               fail_at=2 if i == 3 else None)) for i in range(8)]
        outs = []
        for i, f in enumerate(futs):
            if i == 3:
                with pytest.raises(RuntimeError):
                    f.result(timeout=30)
            else:
                outs.append(f.result(timeout=30))
    assert len(outs) == 7 and ex.max_live >= 2
    assert srv._reserved == 0 and srv._resident_jobs == 0
    assert ("release", "r3", 0) in ex.log
