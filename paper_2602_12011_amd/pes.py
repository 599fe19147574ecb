"""Thin ctypes binding of libpes (the C-ABI in include/pes.h).

Argument marshalling only: every step of the response and likelihood runs in
the library's HIP kernels.  Device memory and streams come from PyTorch
tensors (``tensor.data_ptr()``, ``torch.cuda.current_stream().cuda_stream``).
The library must have been built (``__graft_entry__.build()``); importing
this module without it raises, there is no fallback.
"""
import ctypes as C
import os

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
                ("oms_asd", C.c_double), ("acc_asd", C.c_double)]


class Config(C.Structure):
    _fields_ = [("n_det", C.c_int), ("det", Detector * 3), ("n_bins", C.c_int64),
                ("f0", C.c_double), ("df", C.c_double), ("n_modes", C.c_int),
                ("modes", (C.c_int * 2) * 5)]


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
        ip = C.POINTER(C.c_int)
        L.pes_set_tuning.argtypes = [vp, C.c_int, C.c_int, C.c_int]
        L.pes_get_tuning.argtypes = [vp, ip, ip, ip]
        L.pes_autotune.argtypes = [vp, vp, C.c_int64, vp, C.POINTER(C.c_double), vp]
        L.pes_timing.argtypes = [vp, C.c_int]
        L.pes_timing_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.pes_strerror.argtypes = [C.c_int]
        L.pes_strerror.restype = C.c_char_p
        L.pes_last_error.argtypes = [vp]
        L.pes_last_error.restype = C.c_char_p
        for name in ("pes_create", "pes_destroy", "pes_reserve", "pes_set_data",
                     "pes_response", "pes_loglike", "pes_timing", "pes_timing_read",
                     "pes_set_tuning", "pes_get_tuning", "pes_autotune"):
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
                            float(d["oms_asd"]), float(d["acc_asd"]))
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


# C-ABI names, for callers that prefer the flat interface.
def pes_create(cfg):
    return Context(cfg)


def pes_set_data(ctx, d, stream=None):
    ctx.set_data(d, stream)


def pes_response(ctx, theta, out=None, stream=None):
    return ctx.response(theta, out, stream)


def pes_loglike(ctx, theta, out=None, stream=None):
    return ctx.loglike(theta, out, stream)


def pes_destroy(ctx):
    ctx.close()
