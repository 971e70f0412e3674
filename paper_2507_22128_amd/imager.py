"""ctypes binding of ``libimager.so`` (C-ABI in ``include/imager.h``).

Argument marshalling only: every step runs in the library's HIP kernels.
Device buffers are torch CUDA tensors; the handle runs on the torch stream
that is current when it is created, so library work and torch work are
ordered on one stream.  There is no CPU fallback: without the built
library every call raises.
"""

import ctypes
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libimager.so")
_LIB = None

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ENOTIMPL = range(6)
C64, C128 = 0, 1
WEIGHT_NATURAL, WEIGHT_UNIFORM = 0, 1
PART_LOW, PART_HIGH = 0, 1
DEGRID_COMPOSITE = 1
GRID_DIRTY, GRID_UNNORMALIZED = 0, 1
COMBINE_EXCHANGE, COMBINE_FINAL = 0, 1

_STATUS = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ESTATE", 5: "ENOTIMPL"}


class ImagerError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (_STATUS.get(code, code), msg))
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [("n_pix", ctypes.c_int32), ("cell_rad", ctypes.c_double),
                ("support", ctypes.c_int32), ("es_beta", ctypes.c_double),
                ("weighting", ctypes.c_int32), ("n_partitions", ctypes.c_int32),
                ("ell_pix", ctypes.c_double), ("delta_pix", ctypes.c_double),
                ("tile", ctypes.c_int32), ("chunk", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("hbm_budget", ctypes.c_size_t), ("stream", ctypes.c_void_p),
                ("autotune", ctypes.c_int32), ("tolerance", ctypes.c_double)]


class Vis(ctypes.Structure):
    _fields_ = [("n_vis", ctypes.c_int64), ("freq_hz", ctypes.c_double),
                ("uvw", ctypes.c_void_p), ("vis", ctypes.c_void_p), ("vis_dtype", ctypes.c_int32),
                ("weight", ctypes.c_void_p), ("flag", ctypes.c_void_p),
                ("on_device", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("n_pix", ctypes.c_int32), ("n_grid", ctypes.c_int32),
                ("support", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("n_partitions", ctypes.c_int32), ("cell_rad", ctypes.c_double),
                ("es_beta", ctypes.c_double), ("ell_pix", ctypes.c_double),
                ("delta_pix", ctypes.c_double), ("n_valid", ctypes.c_int64),
                ("n_vis", ctypes.c_int64 * 2), ("n_chunks", ctypes.c_int64 * 2),
                ("sum_w", ctypes.c_double * 2), ("device_bytes", ctypes.c_size_t),
                ("create_ms", ctypes.c_double), ("chunk", ctypes.c_int32),
                ("device_peak_bytes", ctypes.c_size_t)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("n_members", ctypes.c_int32), ("support", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("chunk", ctypes.c_int32), ("n_vis", ctypes.c_int64),
                ("n_chunks", ctypes.c_int64), ("graph_ready", ctypes.c_int32),
                ("n_sets", ctypes.c_int32)]


BATCH_GRAPH, BATCH_LOOP = 1, 2


_P = ctypes.c_void_p
_I = ctypes.c_int32
_D = ctypes.c_double
_SIGS = {
    "imager_create": [ctypes.POINTER(Config), ctypes.POINTER(Vis), ctypes.POINTER(_P)],
    "imager_destroy": [_P],
    "imager_info": [_P, ctypes.POINTER(Info)],
    "imager_vis_index": [_P, _I, _P],
    "imager_vis_weight": [_P, _I, _P],
    "imager_degrid": [_P, _I, _P, _P],
    "imager_grid": [_P, _I, _P, _P, _I],
    "imager_psf": [_P, _I, _P],
    "imager_major_cycle": [_P, _I, _P, _P, _D, _D, _P, _P, _I],
    "imager_major_cycle_nodes": [_P, _P, _P, _P, _P, _P, _P, _I],
    "imager_composed_psf": [_P, _I, _D, _D, _P],
    "imager_minor_cycle_msclean": [_P, _I, _P, _P, _P, _P, _P, _P, _P, _P],
    "imager_minor_cycle_msclean_static": [_P, _I, _P, _P, _P, _P, _P, _P, _P, _P],
    "imager_reconstruct_msclean": [_P, _I, _P, _P, _P, _P, _P],
    "imager_minor_cycle_fista": [_P, _I, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P],
    "imager_reconstruct_fista": [_P, _I, _P, _P, _P, _P, _P, _P, _P],
    "imager_combine_partitions": [_P, _I, _P, _P, _D, _D, _P, _P],
    "imager_set_timing": [_P, _I],
    "imager_get_timing": [_P, _P],
    "imager_sync": [_P],
    "imager_tune_log": [_P, _I, _P, _P, _P, _P],
    "imager_footprint": [ctypes.POINTER(Config), ctypes.c_int64, _I, _I, _I, _P, _P],
    "imager_set_chunk": [_P, _I],
    "imager_batch_create": [_P, _I, ctypes.POINTER(_P)],
    "imager_batch_destroy": [_P],
    "imager_batch_info": [_P, ctypes.POINTER(BatchInfo)],
    "imager_batch_major_cycle": [_P, _P, _P, _I],
    "imager_batch_autotune": [_P, _P, _I, _I, _P, _P],
    "imager_batch_set_bytes": [_P, ctypes.c_uint64],
}

MAX_SCALES = 8


class MsCleanParams(ctypes.Structure):
    _fields_ = [("n_scales", ctypes.c_int32), ("scales", ctypes.c_double * MAX_SCALES),
                ("active_mask", ctypes.c_uint32), ("gain", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("threshold", ctypes.c_double),
                ("bias_slope", ctypes.c_double), ("own_scales_only", ctypes.c_int32),
                ("first_cycle", ctypes.c_int32)]


COMPONENT_DTYPE = np.dtype([("scale", "<i4"), ("iy", "<i4"), ("ix", "<i4"), ("reserved", "<i4"),
                            ("amp", "<f8")])


def msclean_params(scales, gain=0.1, niter=2000, threshold=0.0, bias_slope=0.6, active=None,
                   own_scales_only=False, first_cycle=0):
    if not 1 <= len(scales) <= MAX_SCALES:
        raise ImagerError(EINVAL, "between 1 and %d scales" % MAX_SCALES)
    p = MsCleanParams()
    p.n_scales = len(scales)
    for i, sc in enumerate(scales):
        p.scales[i] = float(sc)
    p.active_mask = 0 if active is None else sum(1 << int(i) for i in active)
    p.gain = float(gain)
    p.max_iter = int(niter)
    p.threshold = float(threshold)
    p.bias_slope = float(bias_slope)
    p.own_scales_only = 1 if own_scales_only else 0
    p.first_cycle = int(first_cycle)
    return p


class FistaParams(ctypes.Structure):
    _fields_ = [("vanishing", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("n_iter", ctypes.c_int32), ("power_iters", ctypes.c_int32),
                ("lam", ctypes.c_double), ("lambda_frac", ctypes.c_double),
                ("gamma_n", ctypes.c_double), ("serial", ctypes.c_int32),
                ("first_cycle", ctypes.c_int32), ("dictionary", ctypes.c_int32)]


def fista_params(vanishing=8, levels=3, n_iter=200, power_iters=30, lam=0.0, lam_frac=1e-3,
                 gamma_n=0.0, serial=False, first_cycle=0, dictionary=False):
    p = FistaParams()
    p.vanishing, p.levels, p.n_iter, p.power_iters = int(vanishing), int(levels), int(n_iter), \
        int(power_iters)
    p.lam, p.lambda_frac, p.gamma_n = float(lam), float(lam_frac), float(gamma_n)
    p.serial = 1 if serial else 0
    p.first_cycle = int(first_cycle)
    p.dictionary = 1 if dictionary else 0
    return p


N_STAGES = 5
STAGES = ("model_fft", "degrid_grid", "flush", "residual_fft", "compose")


class Timing(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int64), ("ms", ctypes.c_double * N_STAGES)]


def library_path():
    return _LIB_PATH


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(_LIB_PATH):
            raise ImagerError(EINVAL, "libimager.so is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(_LIB_PATH)
        for name, args in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        for name in ("imager_last_error", "imager_batch_last_error"):
            fn = getattr(L, name)
            fn.argtypes = [_P]
            fn.restype = ctypes.c_char_p
        _LIB = L
    return _LIB


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev_f32(t, shape, torch):
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and tuple(t.shape) == shape):
        raise ImagerError(EINVAL, "expected a contiguous cuda float32 tensor of shape %s" % (shape,))
    return t


class Imager:
    """One handle: the visibilities of one data set, sorted and binned per
    partition, plus PSFs and work buffers, resident on the current GPU."""

    def __init__(self, handle, info, stream):
        self._h = handle
        self.info = info
        self._stream = stream

    # ------------------------------------------------------------ lifetime
    @classmethod
    def create(cls, data=None, *, uvw=None, vis=None, freq_hz=None, cell=None, n_pix=None,
               weight=None, flag=None, weighting="uniform", n_partitions=1, ell=-1.0, delta=1.0,
               support=8, beta=0.0, tile=0, chunk=0, hbm_budget=0, stream=None,
               autotune=False, tolerance=0.0):
        """Build a handle from host numpy arrays or cuda tensors.  ``data`` may be
        a dict from ``synth.make`` supplying uvw, vis, freq_hz, cell, n_pix.
        ``support=0`` with ``tolerance > 0`` picks the support for that accuracy;
        ``autotune`` times the candidate tiles / chunk caps left at 0."""
        import torch
        if data is not None:
            uvw = data["uvw"] if uvw is None else uvw
            vis = data["vis"] if vis is None else vis
            freq_hz = data["freq_hz"] if freq_hz is None else freq_hz
            cell = data["cell"] if cell is None else cell
            n_pix = data["n_img"] if n_pix is None else n_pix
        L = lib()
        if stream is None:
            stream = torch.cuda.current_stream()
        keep = []
        on_dev = isinstance(uvw, torch.Tensor) and uvw.is_cuda

        def hostbuf(a, dtype):
            a = np.ascontiguousarray(a, dtype=dtype)
            keep.append(a)
            return ctypes.c_void_p(a.ctypes.data)

        v = Vis()
        if on_dev:
            for t in (uvw, vis, weight, flag):
                if t is not None:
                    assert t.is_cuda and t.is_contiguous()
                    keep.append(t)
            v.n_vis = uvw.shape[0]
            v.uvw = uvw.data_ptr()
            v.vis = vis.data_ptr()
            v.vis_dtype = C128 if vis.dtype == torch.complex128 else C64
            v.weight = None if weight is None else weight.data_ptr()
            v.flag = None if flag is None else flag.data_ptr()
            v.on_device = 1
        else:
            vis = np.asarray(vis)
            v.n_vis = len(vis)
            v.uvw = hostbuf(uvw, np.float64)
            c128 = vis.dtype == np.complex128
            v.vis = hostbuf(vis, np.complex128 if c128 else np.complex64)
            v.vis_dtype = C128 if c128 else C64
            v.weight = None if weight is None else hostbuf(weight, np.float32)
            v.flag = None if flag is None else hostbuf(flag, np.uint8)
            v.on_device = 0
        v.freq_hz = float(freq_hz)
        c = Config()
        c.n_pix = int(n_pix)
        c.cell_rad = float(cell)
        c.support = int(support)
        c.es_beta = float(beta)
        c.weighting = WEIGHT_UNIFORM if weighting == "uniform" else WEIGHT_NATURAL
        c.n_partitions = int(n_partitions)
        c.ell_pix = -1.0 if ell is None else float(ell)
        c.delta_pix = float(delta)
        c.tile = int(tile)
        c.chunk = int(chunk)
        c.flags = 0
        c.hbm_budget = int(hbm_budget)
        c.stream = ctypes.c_void_p(stream.cuda_stream)
        c.autotune = 1 if autotune else 0
        c.tolerance = float(tolerance)
        h = ctypes.c_void_p()
        st = L.imager_create(ctypes.byref(c), ctypes.byref(v), ctypes.byref(h))
        if st != OK:
            raise ImagerError(st, L.imager_last_error(None).decode())
        info = Info()
        L.imager_info(h, ctypes.byref(info))
        return cls(h, info, stream)

    def destroy(self):
        if self._h is not None:
            lib().imager_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def _check(self, st):
        if st != OK:
            raise ImagerError(st, lib().imager_last_error(self._h).decode())

    # ------------------------------------------------------------ properties
    @property
    def n_pix(self):
        return self.info.n_pix

    def n_vis(self, part):
        return self.info.n_vis[part]

    def sum_w(self, part):
        return self.info.sum_w[part]

    def _empty(self, shape, dtype):
        import torch
        return torch.empty(shape, dtype=getattr(torch, dtype), device="cuda")

    # ------------------------------------------------------------ calls
    def tune_log(self):
        """[(tile, chunk, ms)] of the create-time autotuner."""
        n = ctypes.c_int32()
        self._check(lib().imager_tune_log(self._h, 0, None, None, None, ctypes.byref(n)))
        k = n.value
        t, c, m = np.zeros(k, np.int32), np.zeros(k, np.int32), np.zeros(k, np.float32)
        if k:
            self._check(lib().imager_tune_log(self._h, k, t.ctypes.data_as(_P), c.ctypes.data_as(_P),
                                              m.ctypes.data_as(_P), ctypes.byref(n)))
        return [(int(a), int(b), float(x)) for a, b, x in zip(t, c, m)]

    def set_chunk(self, chunk):
        self._check(lib().imager_set_chunk(self._h, int(chunk)))
        self.refresh_info()

    def refresh_info(self):
        info = Info()
        lib().imager_info(self._h, ctypes.byref(info))
        self.info = info

    def vis_index(self, part):
        out = np.empty(self.n_vis(part), np.int64)
        self._check(lib().imager_vis_index(self._h, part, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def vis_weight(self, part):
        out = np.empty(self.n_vis(part), np.float32)
        self._check(lib().imager_vis_weight(self._h, part, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def degrid(self, part, model, out=None):
        import torch
        n = self.n_pix
        _dev_f32(model, (n, n), torch)
        out = self._empty((self.n_vis(part),), "complex64") if out is None else out
        self._check(lib().imager_degrid(self._h, part, _ptr(model), _ptr(out)))
        return out

    def grid(self, part, vis, mode=GRID_DIRTY, out=None):
        import torch
        n = self.n_pix
        if not (vis.is_cuda and vis.dtype == torch.complex64 and vis.is_contiguous()
                and vis.shape == (self.n_vis(part),)):
            raise ImagerError(EINVAL, "vis must be a contiguous cuda complex64 member vector")
        out = self._empty((n, n), "float32") if out is None else out
        self._check(lib().imager_grid(self._h, part, _ptr(vis), _ptr(out), mode))
        return out

    def psf(self, part, out=None):
        n2 = 2 * self.n_pix
        out = self._empty((n2, n2), "float32") if out is None else out
        self._check(lib().imager_psf(self._h, part, _ptr(out)))
        return out

    def major_cycle(self, part, model, rho_other=None, gamma=1.0, mu=0.0, composite=False,
                    out=None, local_out=None):
        import torch
        n = self.n_pix
        _dev_f32(model, (n, n), torch)
        if rho_other is not None:
            _dev_f32(rho_other, (n, n), torch)
        out = self._empty((n, n), "float32") if out is None else out
        self._check(lib().imager_major_cycle(
            self._h, part, _ptr(model), _ptr(rho_other), float(gamma), float(mu), _ptr(out),
            _ptr(local_out), DEGRID_COMPOSITE if composite else 0))
        return out

    def major_cycle_nodes(self, models, rho_others=None, gammas=None, mus=None, composite=False,
                          outs=None, local_outs=None):
        """All nodes' major cycles at once (concurrent on the device); lists
        with one entry per partition.  Returns the list of outputs."""
        import torch
        n, k = self.n_pix, self.info.n_partitions
        for m in models:
            _dev_f32(m, (n, n), torch)
        outs = [self._empty((n, n), "float32") for _ in range(k)] if outs is None else outs
        gammas = [1.0] * k if gammas is None else gammas
        mus = [0.0] * k if mus is None else mus
        arr = lambda ts: (ctypes.c_void_p * k)(*[None if t is None else t.data_ptr() for t in ts])
        dbl = lambda xs: (ctypes.c_double * k)(*[float(x) for x in xs])
        if rho_others is not None:
            for r in rho_others:
                _dev_f32(r, (n, n), torch)
        self._check(lib().imager_major_cycle_nodes(
            self._h, arr(models), None if rho_others is None else arr(rho_others), dbl(gammas),
            dbl(mus), arr(outs), None if local_outs is None else arr(local_outs),
            DEGRID_COMPOSITE if composite else 0))
        return outs

    def composed_psf(self, part, gamma, mu, out=None):
        n2 = 2 * self.n_pix
        out = self._empty((n2, n2), "float32") if out is None else out
        self._check(lib().imager_composed_psf(self._h, part, float(gamma), float(mu), _ptr(out)))
        return out

    def exchange(self, delta_low, delta_high, rho_for_low, rho_for_high):
        """rho_for_low += Gamma_H (dH - dL); rho_for_high += Gamma_L (dL - dH)."""
        self._check(lib().imager_combine_partitions(
            self._h, COMBINE_EXCHANGE, _ptr(delta_low), _ptr(delta_high), 0.0, 0.0,
            _ptr(rho_for_low), _ptr(rho_for_high)))

    def combine_final(self, a, b, wa=0.5, wb=0.5, out=None):
        n = self.n_pix
        out = self._empty((n, n), "float64") if out is None else out
        self._check(lib().imager_combine_partitions(
            self._h, COMBINE_FINAL, _ptr(a), _ptr(b), float(wa), float(wb), _ptr(out), None))
        return out

    def minor_cycle_msclean(self, part, dirty, psf, scales, gain=0.1, niter=2000, threshold=0.0,
                            bias_slope=0.6, active=None, own_scales_only=False, model_accum=None,
                            want_residual=True, static=False):
        """Multi-scale CLEAN of one node (synchronous).  Returns (model_delta,
        components (numpy structured array), residual or None).  With
        ``static`` the library's non-allocating entry point is called
        (imager_minor_cycle_msclean_static)."""
        import torch
        n = self.n_pix
        _dev_f32(dirty, (n, n), torch)
        _dev_f32(psf, (2 * n, 2 * n), torch)
        prm = msclean_params(scales, gain, niter, threshold, bias_slope, active, own_scales_only)
        delta = self._empty((n, n), "float32")
        resid = self._empty((n, n), "float32") if want_residual else None
        comps = torch.empty(max(int(niter), 1) * COMPONENT_DTYPE.itemsize, dtype=torch.uint8,
                            device="cuda")
        cnt = ctypes.c_int32(0)
        fn = (lib().imager_minor_cycle_msclean_static if static
              else lib().imager_minor_cycle_msclean)
        self._check(fn(self._h, part, ctypes.byref(prm), _ptr(dirty), _ptr(psf), _ptr(delta),
                       _ptr(model_accum), _ptr(resid), _ptr(comps), ctypes.byref(cnt)))
        raw = comps[:cnt.value * COMPONENT_DTYPE.itemsize].cpu().numpy()
        return delta, np.frombuffer(raw.tobytes(), dtype=COMPONENT_DTYPE), resid

    def reconstruct_msclean(self, n_cycles, scales, gain=0.1, niter=2000, threshold=0.0,
                            bias_slope=0.6, active=None, models=None, rhos=None, first_cycle=0,
                            final=None):
        """The whole major/minor loop in the library (cycles first_cycle ..
        first_cycle + n_cycles - 1).  Returns (final image (float64), per-node
        models, per-node rho, components per cycle and node)."""
        n, k = self.n_pix, self.info.n_partitions
        prm = msclean_params(scales, gain, niter, threshold, bias_slope, active,
                             first_cycle=first_cycle)
        import torch
        models = [torch.zeros((n, n), device="cuda") for _ in range(k)] if models is None else models
        rhos = [torch.zeros((n, n), device="cuda") for _ in range(k)] if rhos is None else rhos
        final = self._empty((n, n), "float64") if final is None else final
        counts = np.zeros((n_cycles, k), np.int32)
        arr = lambda ts: (ctypes.c_void_p * k)(*[t.data_ptr() for t in ts])
        self._check(lib().imager_reconstruct_msclean(
            self._h, int(n_cycles), ctypes.byref(prm), arr(models), arr(rhos), _ptr(final),
            counts.ctypes.data_as(ctypes.c_void_p)))
        return final, models, rhos, counts

    def minor_cycle_fista(self, part, dirty, power_start, rho_other=None, model_accum=None,
                          want_objective=False, psf=None, **params):
        """Sparsity-regularised minor cycle of one node (synchronous); psf (2N x
        2N) replaces the node's own PSF in H when given.  Returns
        (model_delta, objective per iteration or None, L_hat, lambda)."""
        import torch
        n = self.n_pix
        _dev_f32(dirty, (n, n), torch)
        _dev_f32(power_start, (n, n), torch)
        if psf is not None:
            _dev_f32(psf, (2 * n, 2 * n), torch)
        prm = fista_params(**params)
        delta = self._empty((n, n), "float32")
        obj = self._empty((max(prm.n_iter, 1),), "float64") if want_objective else None
        L, lam = ctypes.c_double(0.0), ctypes.c_double(0.0)
        self._check(lib().imager_minor_cycle_fista(
            self._h, part, ctypes.byref(prm), _ptr(dirty), _ptr(psf), _ptr(rho_other),
            _ptr(power_start),
            _ptr(delta), _ptr(model_accum), _ptr(obj), ctypes.byref(L), ctypes.byref(lam)))
        objective = None if obj is None else obj[:prm.n_iter].cpu().numpy()
        return delta, objective, L.value, lam.value

    def reconstruct_fista(self, n_cycles, power_starts, models=None, rhos=None, final=None,
                          **params):
        """The whole loop with the sparsity-regularised minor cycle (params may
        hold first_cycle).  Returns (final image (float64), models, rhos, L_hat
        and lambda per cycle and node)."""
        import torch
        n, k = self.n_pix, self.info.n_partitions
        prm = fista_params(**params)
        models = [torch.zeros((n, n), device="cuda") for _ in range(k)] if models is None else models
        rhos = [torch.zeros((n, n), device="cuda") for _ in range(k)] if rhos is None else rhos
        final = self._empty((n, n), "float64") if final is None else final
        Ls = np.zeros((n_cycles, k))
        lams = np.zeros((n_cycles, k))
        arr = lambda ts: (ctypes.c_void_p * k)(*[t.data_ptr() for t in ts])
        self._check(lib().imager_reconstruct_fista(
            self._h, int(n_cycles), ctypes.byref(prm), arr(power_starts), arr(models), arr(rhos),
            _ptr(final), Ls.ctypes.data_as(ctypes.c_void_p), lams.ctypes.data_as(ctypes.c_void_p)))
        return final, models, rhos, Ls, lams

    def set_timing(self, enable):
        self._check(lib().imager_set_timing(self._h, 1 if enable else 0))

    def get_timing(self):
        """(cycles, {stage: summed ms}) since the last call; synchronises."""
        t = Timing()
        self._check(lib().imager_get_timing(self._h, ctypes.byref(t)))
        return t.cycles, dict(zip(STAGES, list(t.ms)))

    def sync(self):
        self._check(lib().imager_sync(self._h))


def footprint(n_pix, n_vis, n_partitions=1, support=8, tile=0, chunk=0, autotune=False,
              tolerance=0.0, ell=-1.0, vis_on_host=False, n_scales=0, fista=0):
    """(resident, peak) device bytes of a handle before it is built; fista =
    the number of dictionary bases of a FISTA minor cycle (0: none)."""
    c = Config()
    c.n_pix, c.n_partitions, c.support = int(n_pix), int(n_partitions), int(support)
    c.tile, c.chunk, c.autotune, c.tolerance = int(tile), int(chunk), int(bool(autotune)), \
        float(tolerance)
    c.ell_pix = float(ell)
    r, p = ctypes.c_size_t(), ctypes.c_size_t()
    st = lib().imager_footprint(ctypes.byref(c), int(n_vis), int(bool(vis_on_host)),
                                int(n_scales), int(fista), ctypes.byref(r), ctypes.byref(p))
    if st != OK:
        raise ImagerError(st, "footprint: bad configuration")
    return r.value, p.value


def _ptr_array(ts):
    arr = (ctypes.c_void_p * len(ts))()
    for i, t in enumerate(ts):
        arr[i] = t.data_ptr()
    return arr


class Batch:
    """Major cycles of many single-partition handles (e.g. frequency
    channels) with one fused de/gridding launch over all of them."""

    def __init__(self, members):
        self.members = list(members)
        hs = (ctypes.c_void_p * len(self.members))(*[m._h.value for m in self.members])
        b = ctypes.c_void_p()
        st = lib().imager_batch_create(hs, len(self.members), ctypes.byref(b))
        if st != OK:
            raise ImagerError(st, lib().imager_batch_last_error(None).decode())
        self._b = b

    def _check(self, st):
        if st != OK:
            raise ImagerError(st, lib().imager_batch_last_error(self._b).decode())

    def destroy(self):
        if self._b is not None:
            lib().imager_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def info(self):
        o = BatchInfo()
        self._check(lib().imager_batch_info(self._b, ctypes.byref(o)))
        return o

    def major_cycle(self, models, residuals=None, graph=False, loop=False):
        """residuals[i] = Eq. 2 residual of member i for models[i]."""
        import torch
        assert len(models) == len(self.members)
        for m, t in zip(self.members, models):
            _dev_f32(t, (m.n_pix, m.n_pix), torch)
        if residuals is None:
            residuals = [torch.empty((m.n_pix, m.n_pix), dtype=torch.float32, device="cuda")
                         for m in self.members]
        for m, t in zip(self.members, residuals):
            _dev_f32(t, (m.n_pix, m.n_pix), torch)
        flags = (BATCH_GRAPH if graph else 0) | (BATCH_LOOP if loop else 0)
        self._keep = (models, residuals)
        self._check(lib().imager_batch_major_cycle(self._b, _ptr_array(models),
                                                   _ptr_array(residuals), flags))
        return residuals

    def set_bytes(self, nbytes):
        """Cache budget of a member set (0: default; at least the members'
        total: one set)."""
        self._check(lib().imager_batch_set_bytes(self._b, int(nbytes)))

    def autotune(self, caps=(256, 512, 1024, 2048, 4096), reps=3):
        """Times the fused launch for every chunk cap, applies the fastest;
        returns (chosen, {cap: ms})."""
        caps_a = np.asarray(caps, np.int32)
        ms = np.zeros(len(caps_a), np.float32)
        chosen = ctypes.c_int32()
        self._check(lib().imager_batch_autotune(self._b, caps_a.ctypes.data_as(_P), len(caps_a),
                                                int(reps), ms.ctypes.data_as(_P),
                                                ctypes.byref(chosen)))
        for m in self.members:
            m.refresh_info()
        return int(chosen.value), {int(c): float(x) for c, x in zip(caps_a, ms)}
