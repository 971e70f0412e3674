"""Serving loop: reconstruction requests on one GPU with continuous batching.

A request is one imaging job: a visibility set (uvw, vis, flags, frequency,
cell, image size), a minor-cycle method (multi-scale CLEAN or FISTA, Sections
4.1 and 4.2), a number of major cycles and one or two partitions.  Requests
arrive at any time and wait in FIFO order until their device-memory
footprint fits next to the requests already resident (admission by HBM
footprint: the library's ``imager_footprint`` peak estimate while the handle
is built, then its resident estimate).  Admitted requests keep their handle
(sorted visibilities, PSFs, work areas), models, rho and output on the device
across cycles.  Worker threads take the next due request, run ONE major
cycle of it (Eq. 2, the composition of Eq. 7, the minor cycle, the exchange)
and put it back, so new requests join and finished ones leave at cycle
boundaries (continuous batching), and up to ``workers`` cycles of different
requests run concurrently, each on its own stream.  A request's arithmetic
stays in its own handle and buffers and every kernel is deterministic, so
its result does not depend on what else is in flight, and running its
cycles one call at a time gives the same bits as one library call for all
of them (``first_cycle``).

The scheduling logic is independent of the GPU: ``Server`` drives an
executor (``ImagerExecutor`` here, a fake one in the CPU tests).
"""

import collections
import dataclasses
import threading
import time
from concurrent.futures import Future

from . import imager


@dataclasses.dataclass
class Request:
    uvw: object                 # [M, 3] float64 metres (numpy or cuda tensor)
    vis: object                 # [M] complex64 / complex128
    freq_hz: float
    cell: float
    n_pix: int
    flag: object = None         # [M] uint8, nonzero = flagged
    method: str = "msclean"     # "msclean" or "fista"
    n_cycles: int = 5
    n_partitions: int = 2
    scales: tuple = (0, 4, 12)
    gain: float = 0.1
    niter: int = 500            # msCLEAN components per cycle and node
    fista_iter: int = 50
    power_iters: int = 30
    lam_frac: float = 1e-3
    power_seed: int = 0         # seed of the power-iteration start image
    support: int = 8
    name: str = ""

    @property
    def n_vis(self):
        return int(self.vis.shape[0])

    @property
    def on_host(self):
        return not (hasattr(self.vis, "is_cuda") and self.vis.is_cuda)


@dataclasses.dataclass
class Result:
    name: str
    final: object               # N x N float64 cuda tensor (Section 5.2 combination)
    models: list
    n_valid: int                # unflagged visibilities
    n_cycles: int
    arrival: float
    admitted: float
    finished: float
    footprint: tuple            # (resident, peak) estimate in bytes
    device_bytes: int           # the handle's device memory at the end
    device_peak_bytes: int      # the most it held at once

    @property
    def latency(self):
        return self.finished - self.arrival


class ImagerExecutor:
    """Runs requests through the HIP library, one stream per request."""

    def __init__(self):
        # bring up the device and the library in the constructing thread, so
        # the workers only enqueue work
        import torch
        torch.cuda.init()
        torch.zeros(1, device="cuda")
        torch.cuda.synchronize()
        imager.lib()

    def footprint(self, req):
        resident, peak = imager.footprint(
            req.n_pix, req.n_vis, n_partitions=req.n_partitions, support=req.support,
            vis_on_host=req.on_host, n_scales=len(req.scales) if req.method == "msclean" else 0,
            fista=req.method == "fista")
        # models, rho, start images and the FP64 final image held beside the handle
        extra = (3 * req.n_partitions * 4 + 8) * req.n_pix * req.n_pix
        return resident + extra, peak + extra

    def start(self, req):
        import numpy as np
        import torch
        st = dict(req=req, stream=torch.cuda.Stream())
        with torch.cuda.stream(st["stream"]):
            h = imager.Imager.create(uvw=req.uvw, vis=req.vis, freq_hz=req.freq_hz, cell=req.cell,
                                     n_pix=req.n_pix, flag=req.flag, weighting="uniform",
                                     n_partitions=req.n_partitions, support=req.support)
            n, k = req.n_pix, req.n_partitions
            st["h"] = h
            st["models"] = [torch.zeros((n, n), device="cuda") for _ in range(k)]
            st["rhos"] = [torch.zeros((n, n), device="cuda") for _ in range(k)]
            st["final"] = torch.empty((n, n), dtype=torch.float64, device="cuda")
            if req.method == "fista":
                rng = np.random.default_rng(req.power_seed)
                st["starts"] = [torch.tensor(rng.standard_normal((n, n)), dtype=torch.float32,
                                             device="cuda") for _ in range(k)]
        return st

    def cycle(self, st, k):
        import torch
        req, h = st["req"], st["h"]
        with torch.cuda.stream(st["stream"]):
            if req.method == "msclean":
                h.reconstruct_msclean(1, list(req.scales), gain=req.gain, niter=req.niter,
                                      models=st["models"], rhos=st["rhos"], first_cycle=k,
                                      final=st["final"])
            else:
                h.reconstruct_fista(1, st["starts"], models=st["models"], rhos=st["rhos"],
                                    final=st["final"], n_iter=req.fista_iter,
                                    power_iters=req.power_iters, lam_frac=req.lam_frac,
                                    first_cycle=k)

    def finish(self, st):
        h = st["h"]
        st["stream"].synchronize()
        h.refresh_info()
        return dict(final=st["final"], models=st["models"], n_valid=int(h.info.n_valid),
                    device_bytes=int(h.info.device_bytes),
                    device_peak_bytes=int(h.info.device_peak_bytes))

    def measured_bytes(self, st):
        st["h"].refresh_info()
        return int(st["h"].info.device_bytes)

    def release(self, st):
        h = st.get("h")
        if h is not None:
            h.destroy()
            st["h"] = None


class _Job:
    __slots__ = ("req", "fut", "arrival", "admitted", "state", "next_cycle", "reserved", "fp",
                 "seq", "waited")

    def __init__(self, req, fut, arrival, seq):
        self.req, self.fut, self.arrival, self.seq = req, fut, arrival, seq
        self.admitted = None
        self.state = None
        self.next_cycle = 1
        self.reserved = 0
        self.fp = None
        self.waited = False


class Server:
    """Continuous-batching server.  ``hbm_budget``: device bytes the resident
    requests may hold together; ``workers``: cycles run concurrently."""

    def __init__(self, hbm_budget, workers=4, executor=None, clock=time.perf_counter):
        self.budget = int(hbm_budget)
        self.ex = executor if executor is not None else ImagerExecutor()
        self.clock = clock
        self._cv = threading.Condition()
        self._pending = collections.deque()
        self._ready = collections.deque()
        self._reserved = 0
        self._running = 0
        self._closing = False
        self._seq = 0
        # statistics
        self.max_reserved = 0
        self.max_resident_jobs = 0
        self.max_concurrent_cycles = 0
        self.admission_waits = 0
        self.admit_order = []
        self._resident_jobs = 0
        self._threads = [threading.Thread(target=self._work, name="imager-serve-%d" % i,
                                          daemon=True) for i in range(int(workers))]
        for t in self._threads:
            t.start()

    # ------------------------------------------------------------ client side
    def submit(self, req):
        fut = Future()
        fp = self.ex.footprint(req)
        with self._cv:
            if self._closing:
                raise RuntimeError("server is closed")
            job = _Job(req, fut, self.clock(), self._seq)
            self._seq += 1
            job.fp = fp
            if fp[1] > self.budget:
                fut.set_exception(imager.ImagerError(
                    imager.ENOMEM, "request %r needs %d bytes at peak, the budget is %d"
                    % (req.name, fp[1], self.budget)))
                return fut
            self._pending.append(job)
            self._cv.notify_all()
        return fut

    def close(self, wait=True):
        with self._cv:
            self._closing = True
            self._cv.notify_all()
        if wait:
            for t in self._threads:
                t.join()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------ scheduler
    def _next_task(self):
        """Under the lock: admit the FIFO head if it fits, else advance the
        next resident request by one cycle."""
        if self._pending:
            head = self._pending[0]
            if self._reserved + head.fp[1] <= self.budget:
                self._pending.popleft()
                head.reserved = head.fp[1]
                self._reserve(head.reserved)
                self.admit_order.append(head.req.name)
                self._resident_jobs += 1
                self.max_resident_jobs = max(self.max_resident_jobs, self._resident_jobs)
                return "admit", head
            if not head.waited:  # requests that had to wait for memory
                head.waited = True
                self.admission_waits += 1
        if self._ready:
            return "cycle", self._ready.popleft()
        return None

    def _reserve(self, nbytes):
        self._reserved += nbytes
        self.max_reserved = max(self.max_reserved, self._reserved)

    def _idle(self):
        return not self._pending and not self._ready and self._running == 0

    def _work(self):
        while True:
            with self._cv:
                while True:
                    task = self._next_task()
                    if task is not None:
                        break
                    if self._closing and self._idle():
                        self._cv.notify_all()
                        return
                    self._cv.wait()
                self._running += 1
                self.max_concurrent_cycles = max(self.max_concurrent_cycles, self._running)
            kind, job = task
            try:
                if kind == "admit":
                    job.state = self.ex.start(job.req)
                    job.admitted = self.clock()
                    # after the build only the resident footprint stays reserved
                    keep = max(job.fp[0], self.ex.measured_bytes(job.state))
                    with self._cv:
                        self._reserved += keep - job.reserved
                        job.reserved = keep
                        self._ready.append(job)
                else:
                    self.ex.cycle(job.state, job.next_cycle)
                    job.next_cycle += 1
                    if job.next_cycle > job.req.n_cycles:
                        out = self.ex.finish(job.state)
                        self.ex.release(job.state)
                        res = Result(name=job.req.name, final=out["final"], models=out["models"],
                                     n_valid=out["n_valid"], n_cycles=job.req.n_cycles,
                                     arrival=job.arrival, admitted=job.admitted,
                                     finished=self.clock(), footprint=job.fp,
                                     device_bytes=out["device_bytes"],
                                     device_peak_bytes=out["device_peak_bytes"])
                        with self._cv:
                            self._reserved -= job.reserved
                            self._resident_jobs -= 1
                        job.fut.set_result(res)
                    else:
                        with self._cv:
                            self._ready.append(job)
            except BaseException as e:  # the request fails; the server goes on
                try:
                    if job.state is not None:
                        self.ex.release(job.state)
                finally:
                    with self._cv:
                        self._reserved -= job.reserved
                        self._resident_jobs -= 1
                    job.fut.set_exception(e)
            finally:
                with self._cv:
                    self._running -= 1
                    self._cv.notify_all()


def run_serial(requests):
    """Plain execution for comparison: one request after another, all of its
    cycles in one library call.  Returns [(final, seconds)]."""
    import torch
    out = []
    for req in requests:
        t0 = time.perf_counter()
        h = imager.Imager.create(uvw=req.uvw, vis=req.vis, freq_hz=req.freq_hz, cell=req.cell,
                                 n_pix=req.n_pix, flag=req.flag, weighting="uniform",
                                 n_partitions=req.n_partitions, support=req.support)
        try:
            if req.method == "msclean":
                final = h.reconstruct_msclean(req.n_cycles, list(req.scales), gain=req.gain,
                                              niter=req.niter)[0]
            else:
                import numpy as np
                rng = np.random.default_rng(req.power_seed)
                n = req.n_pix
                starts = [torch.tensor(rng.standard_normal((n, n)), dtype=torch.float32,
                                       device="cuda") for _ in range(req.n_partitions)]
                final = h.reconstruct_fista(req.n_cycles, starts, n_iter=req.fista_iter,
                                            power_iters=req.power_iters,
                                            lam_frac=req.lam_frac)[0]
            torch.cuda.synchronize()
        finally:
            h.destroy()
        out.append((final, time.perf_counter() - t0))
    return out
