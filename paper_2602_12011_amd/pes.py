"""Thin ctypes binding of libpes (the C-ABI in include/pes.h).

Argument marshalling only: every step of the response and likelihood runs in
the library's HIP kernels.  Device memory and streams come from PyTorch
tensors (``tensor.data_ptr()``, ``torch.cuda.current_stream().cuda_stream``).
The library must have been built (``__graft_entry__.build()``); importing
this module without it raises, there is no fallback.
"""
import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpes.so")

KIND = {"lisa": 0, "taiji": 1, "tianqin": 2}


class PesError(RuntimeError):
    pass


class Detector(C.Structure):
    _fields_ = [("kind", C.c_int), ("tdi_gen", C.c_int), ("arm_m", C.c_double),
                ("phase0", C.c_double), ("tq_period_s", C.c_double),
                ("tq_lon", C.c_double), ("tq_lat", C.c_double),
                ("oms_asd", C.c_double), ("acc_asd", C.c_double), ("orbit", C.c_int)]


ORBIT = {"first_order": 0, "kepler": 1}


class Config(C.Structure):
    _fields_ = [("n_det", C.c_int), ("det", Detector * 3), ("n_bins", C.c_int64),
                ("f0", C.c_double), ("df", C.c_double), ("n_modes", C.c_int),
                ("modes", (C.c_int * 2) * 5)]


class Prior(C.Structure):
    _fields_ = [("kind", C.c_int * 11), ("lo", C.c_double * 11), ("hi", C.c_double * 11)]


GRAD_ADJOINT, GRAD_FORWARD = 0, 1
SCHED_QUEUE, SCHED_GRID = 0, 1
PROBE_MODE, PROBE_GEOM, PROBE_LINKS = 0, 1, 2

PRIOR_KIND = {"uniform": 0, "loguniform": 1, "cosine_sin": 2, "sin": 2, "arcsin": 3, "cos": 3,
              "periodic": 4, "fixed": 5}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise PesError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.pes_create.argtypes = [C.POINTER(Config), C.POINTER(vp)]
        L.pes_destroy.argtypes = [vp]
        L.pes_reserve.argtypes = [vp, C.c_int64]
        L.pes_set_data.argtypes = [vp, vp, vp]
        L.pes_response.argtypes = [vp, vp, C.c_int64, vp, vp]
        L.pes_loglike.argtypes = [vp, vp, C.c_int64, vp, vp]
        L.pes_loglike_noalloc.argtypes = [vp, vp, C.c_int64, vp, vp]
        ip = C.POINTER(C.c_int)
        L.pes_set_tuning.argtypes = [vp, C.c_int, C.c_int, C.c_int]
        L.pes_get_tuning.argtypes = [vp, ip, ip, ip]
        L.pes_autotune.argtypes = [vp, vp, C.c_int64, vp, C.POINTER(C.c_double), vp]
        L.pes_grad.argtypes = [vp, vp, C.c_int64, vp, vp, vp]
        L.pes_fisher.argtypes = [vp, vp, C.c_int64, vp, vp]
        L.pes_set_grad_method.argtypes = [vp, C.c_int]
        L.pes_set_schedule.argtypes = [vp, C.c_int]
        L.pes_set_precision.argtypes = [vp, C.c_int]
        L.pes_noise.argtypes = [vp, C.c_uint64, vp, vp]
        L.pes_probe.argtypes = [vp, vp, C.c_int64, C.c_int, vp, vp]
        L.pes_sampler_set_step.argtypes = [vp, C.c_uint64]
        L.pes_flow_create.argtypes = [C.c_uint64, C.POINTER(vp)]
        L.pes_flow_destroy.argtypes = [vp]
        L.pes_flow_num_params.argtypes = []
        L.pes_flow_num_params.restype = C.c_int64
        L.pes_flow_set_params.argtypes = [vp, vp, vp]
        L.pes_flow_get_params.argtypes = [vp, vp, vp]
        L.pes_flow_set_norm.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.pes_flow_set_affine.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.pes_flow_set_temperature.argtypes = [vp, C.c_double]
        L.pes_flow_get_affine.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.pes_flow_forward.argtypes = [vp, vp, C.c_int64, vp, vp, vp]
        L.pes_flow_inverse.argtypes = [vp, vp, C.c_int64, vp, vp, vp]
        L.pes_flow_nll_grad.argtypes = [vp, vp, C.c_int64, vp, vp, vp]
        L.pes_flow_probe.argtypes = [vp, vp, C.c_int64, C.c_int, vp, vp, vp, vp, vp, vp]
        L.pes_flow_adam_step.argtypes = [vp, vp, C.c_float, vp]
        L.pes_flow_fit.argtypes = [vp, vp, C.c_int64, C.c_int64, C.c_int64, C.c_float, C.c_uint64, C.c_int,
                                   vp, vp]
        L.pes_flow_last_error.argtypes = [vp]
        L.pes_flow_last_error.restype = C.c_char_p
        L.pes_sampler_set_flow.argtypes = [vp, vp, C.c_double]
        L.pes_sampler_read_chain.argtypes = [vp, vp, C.POINTER(C.c_int64), vp]
        L.pes_sampler_create.argtypes = [vp, C.POINTER(Prior), C.c_int64, C.c_uint64, C.c_int64,
                                         C.POINTER(vp)]
        L.pes_sampler_destroy.argtypes = [vp]
        L.pes_sampler_set_state.argtypes = [vp, vp, vp]
        L.pes_sampler_step.argtypes = [vp, C.c_int64, vp]
        L.pes_sampler_capture.argtypes = [vp, vp]
        L.pes_sampler_launch.argtypes = [vp, C.c_int64, vp]
        L.pes_sampler_state.argtypes = [vp, vp, vp, vp, C.POINTER(C.c_uint64), vp]
        L.pes_sampler_chain.argtypes = [vp, C.POINTER(vp)]
        L.pes_propose.argtypes = [vp, C.c_int, C.c_int, vp, vp, vp]
        L.pes_philox.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_int64, vp,
                                 vp]
        L.pes_timing.argtypes = [vp, C.c_int]
        L.pes_timing_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.pes_strerror.argtypes = [C.c_int]
        L.pes_strerror.restype = C.c_char_p
        L.pes_last_error.argtypes = [vp]
        L.pes_last_error.restype = C.c_char_p
        for name in ("pes_create", "pes_destroy", "pes_reserve", "pes_set_data",
                     "pes_response", "pes_loglike", "pes_loglike_noalloc", "pes_timing", "pes_timing_read",
                     "pes_set_tuning", "pes_get_tuning", "pes_autotune", "pes_grad", "pes_set_grad_method",
                     "pes_set_schedule", "pes_set_precision", "pes_noise", "pes_probe", "pes_sampler_set_step",
                     "pes_flow_create", "pes_flow_destroy", "pes_flow_set_params", "pes_flow_get_params",
                     "pes_flow_set_norm", "pes_flow_set_affine", "pes_flow_get_affine", "pes_flow_set_temperature", "pes_flow_forward", "pes_flow_inverse",
                     "pes_flow_nll_grad", "pes_flow_probe", "pes_flow_adam_step", "pes_flow_fit", "pes_sampler_set_flow",
                     "pes_sampler_read_chain",
                     "pes_fisher", "pes_sampler_create", "pes_sampler_destroy",
                     "pes_sampler_set_state", "pes_sampler_step", "pes_sampler_capture",
                     "pes_sampler_launch", "pes_sampler_state", "pes_sampler_chain", "pes_propose",
                     "pes_philox"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def make_config(cfg):
    """Workload dict (detectors, n_bins, f0, df, modes) -> Config."""
    c = Config()
    dets = cfg["detectors"]
    c.n_det = len(dets)
    for i, d in enumerate(dets):
        c.det[i] = Detector(KIND[d["kind"]], int(d.get("tdi_gen", 20)), float(d["arm_m"]),
                            float(d.get("phase0", 0.0)), float(d.get("tq_period_s", 0.0)),
                            float(d.get("tq_lon", 0.0)), float(d.get("tq_lat", 0.0)),
                            float(d["oms_asd"]), float(d["acc_asd"]),
                            ORBIT[d.get("orbit", "first_order")])
    c.n_bins = int(cfg["n_bins"])
    c.f0 = float(cfg["f0"])
    c.df = float(cfg["df"])
    c.n_modes = len(cfg["modes"])
    for i, (l, m) in enumerate(cfg["modes"]):
        c.modes[i][0] = l
        c.modes[i][1] = m
    return c


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev_f64(t, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
            and t.is_contiguous()):
        raise PesError(f"{name} must be a contiguous float64 CUDA tensor")
    return C.c_void_p(t.data_ptr())


class Context:
    """Owns a pes_ctx.  Methods mirror the C entry points."""

    def __init__(self, cfg):
        self.cfg = cfg
        self.n_det = len(cfg["detectors"])
        self.n_bins = int(cfg["n_bins"])
        self.n_modes = len(cfg["modes"])
        self._c = make_config(cfg)
        h = C.c_void_p()
        self._check(lib().pes_create(C.byref(self._c), C.byref(h)), "pes_create")
        self.h = h

    def _check(self, rc, name):
        if rc != 0:
            msg = lib().pes_strerror(rc).decode()
            extra = ""
            if getattr(self, "h", None):
                extra = lib().pes_last_error(self.h).decode()
            raise PesError(f"{name}: {msg} ({rc}) {extra}")

    def close(self):
        if getattr(self, "h", None):
            lib().pes_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def timing(self, enable):
        self._check(lib().pes_timing(self.h, int(bool(enable))), "pes_timing")

    def timing_read(self):
        """(summed main-kernel milliseconds, launches) since the last read."""
        ms = C.c_double()
        n = C.c_int64()
        self._check(lib().pes_timing_read(self.h, C.byref(ms), C.byref(n)), "pes_timing_read")
        return ms.value, n.value

    def set_tuning(self, bins_per_lane, walkers_per_group, blocks_per_cu=0):
        self._check(lib().pes_set_tuning(self.h, int(bins_per_lane), int(walkers_per_group),
                                         int(blocks_per_cu)), "pes_set_tuning")

    def get_tuning(self):
        a, b, c = C.c_int(), C.c_int(), C.c_int()
        self._check(lib().pes_get_tuning(self.h, C.byref(a), C.byref(b), C.byref(c)),
                    "pes_get_tuning")
        return dict(bins_per_lane=a.value, walkers_per_group=b.value, blocks_per_cu=c.value)

    def autotune(self, theta, stream=None):
        """Time every tuning candidate on this batch, keep the fastest; returns
        (ms per call, tuning dict)."""
        theta = theta.contiguous()
        out = torch.empty(theta.shape[0], dtype=torch.float64, device=theta.device)
        ms = C.c_double()
        self._check(lib().pes_autotune(self.h, _dev_f64(theta, "theta"), theta.shape[0],
                                       _dev_f64(out, "logl"), C.byref(ms), _stream(stream)),
                    "pes_autotune")
        return ms.value, self.get_tuning()

    def reserve(self, max_walkers):
        self._check(lib().pes_reserve(self.h, int(max_walkers)), "pes_reserve")

    def set_data(self, d, stream=None):
        """d: complex128 or float64 [n_det, 3, n_bins(, 2)] CUDA tensor."""
        if d.dtype == torch.complex128:
            d = torch.view_as_real(d.contiguous())
        d = d.contiguous()
        if tuple(d.shape) != (self.n_det, 3, self.n_bins, 2):
            raise PesError(f"data shape {tuple(d.shape)} != {(self.n_det, 3, self.n_bins, 2)}")
        self._data = d  # keep alive until the copy kernels ran
        self._check(lib().pes_set_data(self.h, _dev_f64(d, "d"), _stream(stream)), "pes_set_data")

    def noise(self, seed, out=None, stream=None):
        """One stationary Gaussian noise realisation [n_det, 3, n_bins, 2] (see pes_noise)."""
        if out is None:
            out = torch.empty((self.n_det, 3, self.n_bins, 2), dtype=torch.float64, device="cuda")
        self._check(lib().pes_noise(self.h, C.c_uint64(seed & (2 ** 64 - 1)), _dev_f64(out, "out"),
                                    _stream(stream)), "pes_noise")
        return out

    def probe(self, theta, stage, stream=None):
        """Stages of the response for testing (see pes_probe): stage "mode",
        "geom" or "links"."""
        theta = theta.contiguous()
        B = theta.shape[0]
        code, shape = {"mode": (PROBE_MODE, (B, self.n_modes, self.n_bins, 3)),
                       "geom": (PROBE_GEOM, (B, self.n_det, self.n_modes, self.n_bins, 12)),
                       "links": (PROBE_LINKS, (B, self.n_det, self.n_bins, 12))}[stage]
        out = torch.empty(shape, dtype=torch.float64, device=theta.device)
        self._check(lib().pes_probe(self.h, _dev_f64(theta, "theta"), B, code, _dev_f64(out, "out"),
                                    _stream(stream)), "pes_probe")
        return out

    def response(self, theta, out=None, stream=None):
        theta = theta.contiguous()
        B = theta.shape[0]
        if out is None:
            out = torch.empty((B, self.n_det, 3, self.n_bins, 2), dtype=torch.float64,
                              device=theta.device)
        self._check(lib().pes_response(self.h, _dev_f64(theta, "theta"), B, _dev_f64(out, "out"),
                                       _stream(stream)), "pes_response")
        return out

    def loglike(self, theta, out=None, stream=None):
        theta = theta.contiguous()
        if theta.dim() != 2 or theta.shape[1] != 11:
            raise PesError("theta must be [B, 11]")
        B = theta.shape[0]
        if out is None:
            out = torch.empty(B, dtype=torch.float64, device=theta.device)
        self._check(lib().pes_loglike(self.h, _dev_f64(theta, "theta"), B, _dev_f64(out, "logl"),
                                      _stream(stream)), "pes_loglike")
        return out

    def loglike_noalloc(self, theta, out=None, stream=None):
        """pes_loglike_noalloc: the same log L in the library's device scratch
        array, with no allocation (the output buffer is the caller's)."""
        theta = theta.contiguous()
        if theta.dim() != 2 or theta.shape[1] != 11:
            raise PesError("theta must be [B, 11]")
        B = theta.shape[0]
        if out is None:
            out = torch.empty(B, dtype=torch.float64, device=theta.device)
        self._check(lib().pes_loglike_noalloc(self.h, _dev_f64(theta, "theta"), B, _dev_f64(out, "logl"),
                                              _stream(stream)), "pes_loglike_noalloc")
        return out

    def grad(self, theta, stream=None):
        """(log L [B], d log L / d theta [B, 11])."""
        theta = theta.contiguous()
        B = theta.shape[0]
        logl = torch.empty(B, dtype=torch.float64, device=theta.device)
        g = torch.empty((B, 11), dtype=torch.float64, device=theta.device)
        self._check(lib().pes_grad(self.h, _dev_f64(theta, "theta"), B, _dev_f64(logl, "logl"),
                                   _dev_f64(g, "grad"), _stream(stream)), "pes_grad")
        return logl, g

    def set_schedule(self, schedule):
        """"queue" (persistent queue over active tiles, the default) or "grid"
        (plain grid over every tile, batch order)."""
        code = {"queue": SCHED_QUEUE, "grid": SCHED_GRID}[schedule]
        self._check(lib().pes_set_schedule(self.h, code), "pes_set_schedule")

    def set_precision(self, bits):
        """64 (default) or 32: the arithmetic of loglike and response (see
        pes_set_precision)."""
        self._check(lib().pes_set_precision(self.h, int(bits)), "pes_set_precision")

    def set_grad_method(self, method):
        """"adjoint" (reverse sweep, the default) or "forward" (tangents)."""
        code = {"adjoint": GRAD_ADJOINT, "forward": GRAD_FORWARD}[method]
        self._check(lib().pes_set_grad_method(self.h, code), "pes_set_grad_method")

    def fisher(self, theta, stream=None):
        """Fisher matrices [B, 11, 11]."""
        theta = theta.contiguous()
        B = theta.shape[0]
        F = torch.empty((B, 11, 11), dtype=torch.float64, device=theta.device)
        self._check(lib().pes_fisher(self.h, _dev_f64(theta, "theta"), B, _dev_f64(F, "F"),
                                     _stream(stream)), "pes_fisher")
        return F


class LogLike(torch.autograd.Function):
    """log L(theta) as a differentiable torch function: forward calls
    pes_loglike, backward calls pes_grad (recomputing the response; nothing
    per bin is stored between the two)."""

    @staticmethod
    def forward(ctx_, theta, pes_ctx):
        ctx_.pes_ctx = pes_ctx
        ctx_.save_for_backward(theta)
        return pes_ctx.loglike(theta.detach())

    @staticmethod
    def backward(ctx_, g_out):
        (theta,) = ctx_.saved_tensors
        _, g = ctx_.pes_ctx.grad(theta.detach())
        return g_out.to(g.dtype)[:, None] * g, None


def loglike_autograd(ctx, theta):
    return LogLike.apply(theta, ctx)


def make_prior(spec):
    """[(kind, lo, hi)] * 11 -> Prior (kinds as in workloads.PRIOR, or 'periodic', 'fixed')."""
    pr = Prior()
    for j, (kind, lo, hi) in enumerate(spec):
        pr.kind[j] = PRIOR_KIND[kind]
        pr.lo[j] = float(lo)
        pr.hi[j] = float(hi)
    return pr


class Sampler:
    """Ensemble DE-MC sampler on a Context (see pes_sampler_create)."""

    def __init__(self, ctx, prior_spec, n_walkers, seed, chain_len=0):
        self.ctx = ctx
        self.B = int(n_walkers)
        self.chain_len = int(chain_len)
        self._prior = make_prior(prior_spec)
        h = C.c_void_p()
        ctx._check(lib().pes_sampler_create(ctx.h, C.byref(self._prior), self.B, C.c_uint64(seed),
                                            self.chain_len, C.byref(h)), "pes_sampler_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().pes_sampler_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_state(self, theta, stream=None):
        theta = theta.contiguous()
        self.ctx._check(lib().pes_sampler_set_state(self.h, _dev_f64(theta, "theta"), _stream(stream)),
                        "pes_sampler_set_state")

    def set_step(self, steps):
        """Resume: the completed-step count of a saved run (see pes_sampler_set_step)."""
        self.ctx._check(lib().pes_sampler_set_step(self.h, C.c_uint64(int(steps))), "pes_sampler_set_step")

    def step(self, n=1, stream=None):
        self.ctx._check(lib().pes_sampler_step(self.h, int(n), _stream(stream)), "pes_sampler_step")

    def capture(self, stream):
        self.ctx._check(lib().pes_sampler_capture(self.h, _stream(stream)), "pes_sampler_capture")

    def launch(self, n=1, stream=None):
        self.ctx._check(lib().pes_sampler_launch(self.h, int(n), _stream(stream)), "pes_sampler_launch")

    def state(self, stream=None):
        dev = torch.device("cuda")
        th = torch.empty((self.B, 11), dtype=torch.float64, device=dev)
        L = torch.empty(self.B, dtype=torch.float64, device=dev)
        acc = torch.empty(self.B, dtype=torch.int64, device=dev)
        steps = C.c_uint64()
        self.ctx._check(lib().pes_sampler_state(self.h, _dev_f64(th, "theta"), _dev_f64(L, "logl"),
                                                C.c_void_p(acc.data_ptr()), C.byref(steps),
                                                _stream(stream)), "pes_sampler_state")
        return th, L, acc, steps.value

    def chain(self):
        p = C.c_void_p()
        self.ctx._check(lib().pes_sampler_chain(self.h, C.byref(p)), "pes_sampler_chain")
        return p.value

    def read_chain(self, stream=None):
        """Stored states, oldest first: [n_states, n_walkers, 11] tensor."""
        out = torch.empty((max(self.chain_len, 1), self.B, 11), dtype=torch.float64, device="cuda")
        n = C.c_int64()
        self.ctx._check(lib().pes_sampler_read_chain(self.h, _dev_f64(out, "out"), C.byref(n), _stream(stream)),
                        "pes_sampler_read_chain")
        return out[:n.value]

    def propose(self, half, kind="de", stream=None):
        """Proposals of the given half: "de", or "flow" (the mixture set by set_flow)."""
        n = self.B // 2 if half == 0 else self.B - self.B // 2
        dev = torch.device("cuda")
        prop = torch.empty((n, 11), dtype=torch.float64, device=dev)
        q = torch.empty(n, dtype=torch.float64, device=dev)
        code = {"de": 0, "flow": 1}[kind]
        self.ctx._check(lib().pes_propose(self.h, code, int(half), _dev_f64(prop, "prop"), _dev_f64(q, "q"),
                                          _stream(stream)), "pes_propose")
        return prop, q

    def set_flow(self, flow, p_flow=0.9):
        """Mix the flow's independence proposal (probability p_flow) with DE; None: DE only."""
        self._flow = flow
        self.ctx._check(lib().pes_sampler_set_flow(self.h, flow.h if flow is not None else None,
                                                   C.c_double(p_flow)), "pes_sampler_set_flow")


class Flow:
    """Affine-coupling flow proposal (see pes_flow_create)."""

    def __init__(self, seed=0):
        h = C.c_void_p()
        rc = lib().pes_flow_create(C.c_uint64(seed), C.byref(h))
        if rc != 0:
            raise PesError(f"pes_flow_create: {lib().pes_strerror(rc).decode()}")
        self.h = h
        self.n_params = int(lib().pes_flow_num_params())

    def _check(self, rc, name):
        if rc != 0:
            raise PesError(f"{name}: {lib().pes_strerror(rc).decode()} "
                           f"({lib().pes_flow_last_error(self.h).decode()})")

    def close(self):
        if getattr(self, "h", None):
            lib().pes_flow_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params, stream=None):
        params = params.contiguous()
        if params.dtype != torch.float32 or params.numel() != self.n_params or not params.is_cuda:
            raise PesError("params must be a CUDA float32 tensor of num_params entries")
        self._check(lib().pes_flow_set_params(self.h, C.c_void_p(params.data_ptr()), _stream(stream)),
                    "pes_flow_set_params")

    def get_params(self, stream=None):
        out = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        self._check(lib().pes_flow_get_params(self.h, C.c_void_p(out.data_ptr()), _stream(stream)),
                    "pes_flow_get_params")
        return out

    def set_norm(self, mu, sigma):
        mu = (C.c_double * 11)(*[float(x) for x in mu])
        sg = (C.c_double * 11)(*[float(x) for x in sigma])
        self._check(lib().pes_flow_set_norm(self.h, mu, sg), "pes_flow_set_norm")

    def set_temperature(self, tau):
        self._check(lib().pes_flow_set_temperature(self.h, C.c_double(tau)), "pes_flow_set_temperature")

    def set_affine(self, mu, L):
        """Whitening u = L^-1 (theta - mu), L lower triangular [11, 11]."""
        mu = (C.c_double * 11)(*[float(x) for x in mu])
        Lf = (C.c_double * 121)(*[float(x) for x in np.asarray(L, dtype=np.float64).ravel()])
        self._check(lib().pes_flow_set_affine(self.h, mu, Lf), "pes_flow_set_affine")

    def get_affine(self):
        mu, L = (C.c_double * 11)(), (C.c_double * 121)()
        self._check(lib().pes_flow_get_affine(self.h, mu, L), "pes_flow_get_affine")
        return np.array(mu[:]), np.array(L[:]).reshape(11, 11)

    def forward(self, theta, stream=None):
        """(z [n, 11], log q(theta) [n])."""
        theta = theta.contiguous()
        n = theta.shape[0]
        z = torch.empty((n, 11), dtype=torch.float64, device=theta.device)
        lq = torch.empty(n, dtype=torch.float64, device=theta.device)
        self._check(lib().pes_flow_forward(self.h, _dev_f64(theta, "theta"), n, _dev_f64(z, "z"),
                                           _dev_f64(lq, "logq"), _stream(stream)), "pes_flow_forward")
        return z, lq

    def inverse(self, z, stream=None):
        """(theta [n, 11], log det [n])."""
        z = z.contiguous()
        n = z.shape[0]
        th = torch.empty((n, 11), dtype=torch.float64, device=z.device)
        ld = torch.empty(n, dtype=torch.float64, device=z.device)
        self._check(lib().pes_flow_inverse(self.h, _dev_f64(z, "z"), n, _dev_f64(th, "theta"),
                                           _dev_f64(ld, "logdet"), _stream(stream)), "pes_flow_inverse")
        return th, ld

    def probe(self, x, inverse=False, stream=None):
        """The forward (theta -> z, log q) or inverse (z -> theta, log det) pass
        with the coupling state at every layer boundary and every layer's
        conditioner stages: (out [n, 11], lq [n], states float32 [9, n, 11],
        running log det float32 [9, n], acts float32 [8, n, 576])."""
        x = x.contiguous()
        n = x.shape[0]
        out = torch.empty((n, 11), dtype=torch.float64, device=x.device)
        lq = torch.empty(n, dtype=torch.float64, device=x.device)
        st = torch.empty((9, n, 11), dtype=torch.float32, device=x.device)
        ld = torch.empty((9, n), dtype=torch.float32, device=x.device)
        acts = torch.empty((8, n, 576), dtype=torch.float32, device=x.device)
        self._check(lib().pes_flow_probe(self.h, _dev_f64(x, "in"), n, 1 if inverse else 0, _dev_f64(out, "out"),
                                         _dev_f64(lq, "lq"), C.c_void_p(st.data_ptr()), C.c_void_p(ld.data_ptr()),
                                         C.c_void_p(acts.data_ptr()), _stream(stream)), "pes_flow_probe")
        return out, lq, st, ld, acts

    def nll_grad(self, theta, stream=None):
        theta = theta.contiguous()
        nll = torch.empty(1, dtype=torch.float64, device=theta.device)
        g = torch.empty(self.n_params, dtype=torch.float32, device=theta.device)
        self._check(lib().pes_flow_nll_grad(self.h, _dev_f64(theta, "theta"), theta.shape[0],
                                            _dev_f64(nll, "nll"), C.c_void_p(g.data_ptr()), _stream(stream)),
                    "pes_flow_nll_grad")
        return nll, g

    def adam_step(self, grad=None, lr=1e-3, stream=None):
        p = C.c_void_p(grad.contiguous().data_ptr()) if grad is not None else None
        self._check(lib().pes_flow_adam_step(self.h, p, C.c_float(lr), _stream(stream)), "pes_flow_adam_step")

    def fit(self, samples, steps, batch, lr=1e-3, seed=0, standardize=True, stream=None):
        """Trains on samples [n, 11] (CUDA float64); returns the per-step NLL."""
        samples = samples.contiguous()
        loss = torch.empty(max(int(steps), 1), dtype=torch.float64, device=samples.device)
        self._check(lib().pes_flow_fit(self.h, _dev_f64(samples, "samples"), samples.shape[0], int(steps),
                                       int(batch), C.c_float(lr), C.c_uint64(seed), int(bool(standardize)),
                                       _dev_f64(loss, "loss"), _stream(stream)), "pes_flow_fit")
        return loss[:int(steps)]


def philox(key, c0, c1, c2, c3, n, stream=None):
    """[n, 4] words (int64 tensor) of Philox4x32-10 for counters (c0 + i, c1, c2, c3)."""
    out = torch.empty((n, 4), dtype=torch.int32, device="cuda")
    rc = lib().pes_philox(C.c_uint64(key), c0, c1, c2, c3, int(n), C.c_void_p(out.data_ptr()),
                          _stream(stream))
    if rc != 0:
        raise PesError(f"pes_philox: {rc}")
    return out.to(torch.int64) & 0xFFFFFFFF


# C-ABI names, for callers that prefer the flat interface.
def pes_create(cfg):
    return Context(cfg)


def pes_set_data(ctx, d, stream=None):
    ctx.set_data(d, stream)


def pes_response(ctx, theta, out=None, stream=None):
    return ctx.response(theta, out, stream)


def pes_loglike(ctx, theta, out=None, stream=None):
    return ctx.loglike(theta, out, stream)


def pes_grad(ctx, theta, stream=None):
    return ctx.grad(theta, stream)


def pes_set_grad_method(ctx, method):
    ctx.set_grad_method(method)


def pes_fisher(ctx, theta, stream=None):
    return ctx.fisher(theta, stream)


def pes_destroy(ctx):
    ctx.close()
