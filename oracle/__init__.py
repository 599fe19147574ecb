"""TEST INFRASTRUCTURE ONLY -- ctypes binding of the CPU oracle.

The oracle (``oracle.cpp``) is a plain, slow FP64 CPU implementation of the
frequency-domain response and Whittle likelihood of arXiv:2602.12011
(Sec. 2.1 response model, Sec. 2.2 parameter estimation).  Only the tests, the
smoke check and the benchmark's CPU-baseline leg may import this module.  It
shares no code with the GPU library and never imports it.

Configurations are passed in as plain dicts (see ``make_config``); arrays are
numpy, complex arrays are numpy complex128.
"""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.cpp")


def build(force=True):
    """Compile liboracle.so with g++ (-O2, no fast-math, OpenMP)."""
    if not force and os.path.exists(_SO):
        return _SO
    tmp = _SO + ".tmp"
    cmd = ["g++", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c++17", "-Wall",
           "-o", tmp, _SRC]
    subprocess.run(cmd, check=True, cwd=_HERE)
    os.replace(tmp, _SO)
    return _SO


class Detector(C.Structure):
    _fields_ = [("kind", C.c_int), ("tdi_gen", C.c_int), ("arm_m", C.c_double),
                ("phase0", C.c_double), ("tq_period_s", C.c_double),
                ("tq_lon", C.c_double), ("tq_lat", C.c_double),
                ("oms_asd", C.c_double), ("acc_asd", C.c_double), ("orbit", C.c_int)]


class Config(C.Structure):
    _fields_ = [("n_det", C.c_int), ("det", Detector * 3), ("n_bins", C.c_int64),
                ("f0", C.c_double), ("df", C.c_double), ("n_modes", C.c_int),
                ("modes", (C.c_int * 2) * 5)]


KIND = {"lisa": 0, "taiji": 1, "tianqin": 2}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = C.CDLL(_SO)
        dp = C.POINTER(C.c_double)
        L.or_loglike.argtypes = [C.POINTER(Config), dp, dp, C.c_int64, C.c_int, C.c_int, dp]
        L.or_grad.argtypes = [C.POINTER(Config), dp, dp, C.c_int64, C.c_int, dp, dp]
        L.or_fisher.argtypes = [C.POINTER(Config), dp, C.c_int64, C.c_int, dp]
        L.or_response.argtypes = [C.POINTER(Config), dp, C.c_int, dp]
        L.or_inner.argtypes = [C.POINTER(Config), dp, dp]
        L.or_inner.restype = C.c_double
        L.or_psd.argtypes = [C.POINTER(Detector), dp, C.c_int64, dp]
        L.or_orbit.argtypes = [C.POINTER(Detector), C.c_double, dp]
        L.or_link_fd.argtypes = [C.c_double, C.c_double, dp, dp, dp, dp, C.c_int]
        L.or_tdi.argtypes = [C.c_double, C.c_double, C.c_int, dp, dp, dp]
        L.or_ylm.argtypes = [C.c_int, C.c_int, C.c_double]
        L.or_ylm.restype = C.c_double
        L.or_pol_coeffs.argtypes = [C.c_int, C.c_int, C.c_double, dp, dp]
        L.or_mode.argtypes = [dp, C.c_int, C.c_int, dp, C.c_int64, dp, dp, dp]
        L.or_sky_basis.argtypes = [C.c_double, C.c_double, C.c_double, dp, dp, dp]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def make_detector(d):
    """dict -> Detector.  Keys: kind ('lisa'|'taiji'|'tianqin'), arm_m,
    phase0, tdi_gen, oms_asd, acc_asd, for TianQin tq_period_s, tq_lon, tq_lat,
    and orbit ('first_order', the default, or 'kepler': exact ellipses)."""
    return Detector(KIND[d["kind"]], int(d.get("tdi_gen", 20)), float(d["arm_m"]),
                    float(d.get("phase0", 0.0)), float(d.get("tq_period_s", 0.0)),
                    float(d.get("tq_lon", 0.0)), float(d.get("tq_lat", 0.0)),
                    float(d["oms_asd"]), float(d["acc_asd"]),
                    {"first_order": 0, "kepler": 1}[d.get("orbit", "first_order")])


def make_config(cfg):
    """dict -> Config.  Keys: detectors (list of dicts), n_bins, f0, df, modes."""
    c = Config()
    dets = cfg["detectors"]
    c.n_det = len(dets)
    for i, d in enumerate(dets):
        c.det[i] = make_detector(d)
    c.n_bins = int(cfg["n_bins"])
    c.f0 = float(cfg["f0"])
    c.df = float(cfg["df"])
    modes = cfg["modes"]
    c.n_modes = len(modes)
    for i, (l, m) in enumerate(modes):
        c.modes[i][0] = l
        c.modes[i][1] = m
    return c


def _check(rc, name):
    if rc != 0:
        raise ValueError(f"{name} failed with status {rc}")


def response(cfg, theta, prec=0):
    """A/E/T of h(theta): complex array [n_det, 3, n_bins]."""
    c = make_config(cfg)
    th = _f64(theta)
    out = np.zeros((c.n_det, 3, c.n_bins, 2))
    _check(lib().or_response(C.byref(c), _p(th), prec, _p(out)), "or_response")
    return out[..., 0] + 1j * out[..., 1]


def _data_arr(data):
    d = np.ascontiguousarray(data, dtype=np.complex128)
    return np.ascontiguousarray(np.stack([d.real, d.imag], axis=-1))


def loglike(cfg, data, theta, prec=0, nthreads=0):
    c = make_config(cfg)
    th = _f64(np.atleast_2d(theta))
    d = _data_arr(data)
    out = np.zeros(th.shape[0])
    _check(lib().or_loglike(C.byref(c), _p(d), _p(th), th.shape[0], prec, nthreads, _p(out)),
           "or_loglike")
    return out


def grad(cfg, data, theta, nthreads=0):
    c = make_config(cfg)
    th = _f64(np.atleast_2d(theta))
    d = _data_arr(data)
    L = np.zeros(th.shape[0])
    g = np.zeros((th.shape[0], 11))
    _check(lib().or_grad(C.byref(c), _p(d), _p(th), th.shape[0], nthreads, _p(L), _p(g)),
           "or_grad")
    return L, g


def fisher(cfg, theta, nthreads=0):
    c = make_config(cfg)
    th = _f64(np.atleast_2d(theta))
    F = np.zeros((th.shape[0], 11, 11))
    _check(lib().or_fisher(C.byref(c), _p(th), th.shape[0], nthreads, _p(F)), "or_fisher")
    return F


def inner(cfg, a, b):
    c = make_config(cfg)
    return lib().or_inner(C.byref(c), _p(_data_arr(a)), _p(_data_arr(b)))


def psd(det, f):
    d = make_detector(det)
    f = _f64(f)
    S = np.zeros((f.size, 3))
    _check(lib().or_psd(C.byref(d), _p(f), f.size, _p(S)), "or_psd")
    return S[:, 0], S[:, 1], S[:, 2]


def orbit(det, t):
    d = make_detector(det)
    x = np.zeros((3, 3))
    _check(lib().or_orbit(C.byref(d), float(t), _p(x)), "or_orbit")
    return x


def link_fd(f, L_s, k, x, H, unit=False):
    """The six links of a static geometry; unit: link directions are the unit
    separations of the spacecraft (exact Kepler orbits) instead of (x_r - x_s)/L."""
    k = _f64(k)
    x = _f64(x)
    H = np.asarray(H, dtype=np.complex128)
    Hr = _f64(np.stack([H.real, H.imag], axis=-1))
    y = np.zeros((3, 3, 2))
    _check(lib().or_link_fd(float(f), float(L_s), _p(k), _p(x), _p(Hr), _p(y), int(bool(unit))), "or_link_fd")
    return y[..., 0] + 1j * y[..., 1]


def tdi(f, L_s, gen, y):
    y = np.asarray(y, dtype=np.complex128)
    yr = _f64(np.stack([y.real, y.imag], axis=-1))
    xyz = np.zeros((3, 2))
    aet = np.zeros((3, 2))
    _check(lib().or_tdi(float(f), float(L_s), int(gen), _p(yr), _p(xyz), _p(aet)), "or_tdi")
    return xyz[:, 0] + 1j * xyz[:, 1], aet[:, 0] + 1j * aet[:, 1]


def ylm(l, m, iota):
    return lib().or_ylm(l, m, float(iota))


def pol_coeffs(l, m, iota):
    kp = np.zeros(2)
    kc = np.zeros(2)
    lib().or_pol_coeffs(l, m, float(iota), _p(kp), _p(kc))
    return kp[0] + 1j * kp[1], kc[0] + 1j * kc[1]


def mode(theta, l, m, f):
    th = _f64(theta)
    f = _f64(np.atleast_1d(f))
    h = np.zeros((f.size, 2))
    psi = np.zeros(f.size)
    tf = np.zeros(f.size)
    _check(lib().or_mode(_p(th), l, m, _p(f), f.size, _p(h), _p(psi), _p(tf)), "or_mode")
    return h[:, 0] + 1j * h[:, 1], psi, tf


def sky_basis(lam, beta, psi):
    k = np.zeros(3)
    ep = np.zeros((3, 3))
    ec = np.zeros((3, 3))
    lib().or_sky_basis(float(lam), float(beta), float(psi), _p(k), _p(ep), _p(ec))
    return k, ep, ec
