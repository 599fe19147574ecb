"""The single-precision response and log-likelihood (pes_set_precision(ctx, 32))
against the FP64 oracle, with a tolerance derived from the FP32 arithmetic, on
the first-order orbit and (kep_* cases) on exact Kepler ellipses, whose orbit
series the FP32 kernels sum in FP32 (13 terms each; the Roemer delay from the
centroid's series stays within the dR below, |k.c| <= (1 + e) AU/c).

With u = 2^-24 the unit roundoff of FP32, a channel value at frequency f of a
detector with arm L (light-seconds) carries a relative error of at most

    eps(f) = 2 pi f dR + 200 u + 20 u / (pi f L),

  dR = 5 u AU/c   the timing error of the Roemer delay k.R (|k.R| <= AU/c, two
                  FP32 products of the orbit's sine and cosine and a sum);
  200 u           the rest of the FP32 chain (amplitude, projections, links);
  20 u / (pi f L) the cancellation of forward and backward links in the TDI
                  differences, which leaves a fraction ~ pi f L of the link
                  magnitude (the FP64 path has the same structure 2^29 times
                  smaller).
The T channel, which cancels as (f L)^3 against A and E, may also be off by
20 u / (pi f L) of the A/E magnitude at the same bin.

Responses are compared element by element: |h32 - h| <= eps(f) |h| + 1e-6
max|h|.  A log-likelihood error is, to first order, Re <d - h|dh>, so each
walker's is bounded by sum over bins and channels of w |d - h| eps(f) |h|
(w = 4 df / S the channel weight), computed from the oracle's own response;
the test allows twice that plus the FP64 tolerance 1e-9 max(|L|, <d|d>/2).
"""
import math

import numpy as np
import pytest

from paper_2602_12011_amd import workloads as W

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
C_LIGHT = 299792458.0
AU_C = 149597870700.0 / C_LIGHT


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.fixture(scope="module")
def pes():
    from paper_2602_12011_amd import pes as P
    return P


def _cfg(name, n_bins=None, dets=None, kepler=False):
    c = W.config(name, n_bins=n_bins)
    if dets is not None:
        c["detectors"] = dets
    if kepler:   # heliocentric detectors on exact Kepler ellipses (TianQin stays geocentric)
        c["detectors"] = [d if d["kind"] == "tianqin" else dict(d, orbit="kepler") for d in c["detectors"]]
    return c


def _eps(f, det):
    L = det["arm_m"] / C_LIGHT
    return 2.0 * math.pi * f * 5.0 * U32 * AU_C + 200.0 * U32 + 20.0 * U32 / (math.pi * f * L)


CASES = {
    # name: (config, walkers, flat prior)
    "cfg0_full": (lambda: _cfg("cfg0"), 400, True),
    "hm_ragged": (lambda: _cfg("cfg1", n_bins=20000 + 37), 32, False),
    "net_ragged": (lambda: _cfg("cfg2", n_bins=9000 + 5), 16, False),
    "tdi15_hm": (lambda: _cfg("cfg1", n_bins=4096 + 255, dets=[dict(W.LISA, tdi_gen=15)]), 12, False),
    "pe_long_sinc": (lambda: W.config("pehm"), 12, False),
    "kep_hm_ragged": (lambda: _cfg("cfg1", n_bins=20000 + 37, kepler=True), 32, False),
    "kep_net_ragged": (lambda: _cfg("cfg2", n_bins=9000 + 5, kepler=True), 16, False),
    "kep_pe_long_sinc": (lambda: _cfg("pehm", kepler=True), 12, False),
}


def _freqs(cfg):
    return cfg["f0"] + np.arange(cfg["n_bins"]) * cfg["df"]


@pytest.mark.parametrize("case", ["cfg0_full", "hm_ragged", "net_ragged", "tdi15_hm", "pe_long_sinc",
                                  "kep_hm_ragged", "kep_net_ragged", "kep_pe_long_sinc"])
def test_response_fp32(orc, torch_dev, pes, case):
    torch = torch_dev
    cfg = CASES[case][0]()
    th = np.vstack([W.THETA_PE if case.endswith("pe_long_sinc") else W.THETA0,
                    W.draw_walkers(3, stream=21, flat=CASES[case][2])])
    if case.endswith("pe_long_sinc"):
        th[1, 0] = 1.0e5            # a light walker reaches the long-sinc bins
    print(f"[fp32] response {case}: n_bins={cfg['n_bins']} dets={len(cfg['detectors'])}", flush=True)
    ctx = pes.Context(cfg)
    ctx.set_precision(32)
    out = ctx.response(torch.from_numpy(th).to("cuda")).cpu().numpy()
    ctx.close()
    h32 = out[..., 0] + 1j * out[..., 1]
    f = _freqs(cfg)
    worst = 0.0
    for b in range(th.shape[0]):
        h_or = orc.response(cfg, th[b], prec=1)
        for det, dd in enumerate(cfg["detectors"]):
            eps = _eps(f, dd)
            ae = np.sqrt(np.abs(h_or[det, 0]) ** 2 + np.abs(h_or[det, 1]) ** 2)
            for c in range(3):
                ref = h_or[det, c]
                tol = eps * np.abs(ref) + 1e-6 * np.abs(ref).max()
                if c == 2:
                    tol = tol + 20.0 * U32 / (math.pi * f * dd["arm_m"] / C_LIGHT) * ae
                err = np.abs(h32[b, det, c] - ref)
                if np.abs(ref).max() > 0:
                    worst = max(worst, float((err / tol).max()))
                assert np.all(err <= tol), (case, b, det, c, float((err / tol).max()))
    # the relative error actually reached, for the record
    print(f"[fp32] response {case}: worst error / bound {worst:.3f}", flush=True)


def _loglike_bound(orc, cfg, d, th):
    """Per walker: sum_{det, c, k} w |d - h| eps(f_k) |h| from the oracle's response."""
    f = _freqs(cfg)
    bound = np.zeros(th.shape[0])
    for b in range(th.shape[0]):
        h = orc.response(cfg, th[b])
        if not np.all(np.isfinite(h)):
            bound[b] = np.inf
            continue
        for det, dd in enumerate(cfg["detectors"]):
            SA, SE, ST = orc.psd(dd, f)
            eps = _eps(f, dd)
            for c, S in enumerate((SA, SE, ST)):
                w = np.where(S > 0, 4.0 * cfg["df"] / np.where(S > 0, S, 1.0), 0.0)
                bound[b] += np.sum(w * np.abs(d[det, c] - h[det, c]) * eps * np.abs(h[det, c]))
    return bound


@pytest.mark.parametrize("case", list(CASES))
def test_loglike_fp32(orc, torch_dev, pes, case):
    torch = torch_dev
    mk, B, flat = CASES[case]
    cfg = mk()
    inj = W.THETA_PE if case.endswith("pe_long_sinc") else W.THETA0
    d = orc.response(cfg, inj)
    th = np.vstack([inj, W.draw_walkers(B - 1, stream=11, flat=flat)])
    print(f"[fp32] loglike {case}: n_bins={cfg['n_bins']} dets={len(cfg['detectors'])} B={B}", flush=True)
    ctx = pes.Context(cfg)
    ctx.set_data(torch.from_numpy(np.ascontiguousarray(d)).to("cuda"))
    tht = torch.from_numpy(th).to("cuda")
    L64 = ctx.loglike(tht).cpu().numpy()
    ctx.set_precision(32)
    Ls = []
    for bpl in (1, 2):
        ctx.set_tuning(bpl, 16, 0)
        Ls.append(ctx.loglike(tht).cpu().numpy())
    Ln = ctx.loglike_noalloc(tht).cpu().numpy()   # the same kernels in the library's scratch array
    ctx.close()
    assert np.array_equal(Ln, Ls[1])
    L_or = orc.loglike(cfg, d, th)
    sigma = 0.5 * orc.inner(cfg, d, d)
    bound = 2.0 * _loglike_bound(orc, cfg, d, th) + 1e-9 * np.maximum(np.abs(L_or), sigma)
    fin = np.isfinite(L_or)
    for L in Ls:
        assert np.array_equal(np.isfinite(L), fin)
        err = np.abs(L[fin] - L_or[fin])
        w = int(np.argmax(err / bound[fin]))
        assert np.all(err <= bound[fin]), (case, w, err[w], bound[fin][w])
        rel = err / np.maximum(np.abs(L_or[fin]), sigma)
        print(f"[fp32] loglike {case}: worst |dL| / bound {float((err / bound[fin]).max()):.3f}, "
              f"worst |dL| / max(|L|, <d|d>/2) {float(rel.max()):.2e} "
              f"(FP64 path {float((np.abs(L64[fin] - L_or[fin]) / np.maximum(np.abs(L_or[fin]), sigma)).max()):.1e})",
              flush=True)
    # both bin-per-lane variants of the FP32 kernel evaluate the same terms
    assert np.allclose(Ls[0], Ls[1], rtol=1e-12, atol=1e-9 * sigma)


@pytest.mark.parametrize("kepler", [False, True])
def test_fp32_full_size_sampled(orc, torch_dev, pes, kepler):
    """The benchmark's FP32 launches (4096 walkers, 2^20 bins, five modes, on
    the first-order orbit and on exact Kepler ellipses) on 8 walkers at evenly
    spaced ranks of the mass order, against the oracle with the derived bound
    above."""
    torch = torch_dev
    cfg = _cfg("cfg1", kepler=kepler)
    B = cfg["walkers"]
    print(f"[fp32] full size: kepler={kepler} B={B} n_bins={cfg['n_bins']}", flush=True)
    d = orc.response(cfg, W.THETA0)
    th = W.draw_walkers(B, stream=1)
    ctx = pes.Context(cfg)
    ctx.set_data(torch.from_numpy(np.ascontiguousarray(d)).to("cuda"))
    ctx.set_precision(32)
    tht = torch.from_numpy(th).to("cuda")
    ctx.autotune(tht)
    L = ctx.loglike(tht).cpu().numpy()
    ctx.close()
    assert np.all(np.isfinite(L)) and np.all(L <= 0)
    order = np.argsort(th[:, 0], kind="stable")
    idx = np.unique(order[np.linspace(0, B - 1, 8).round().astype(int)])
    L_or = orc.loglike(cfg, d, th[idx])
    sigma = 0.5 * orc.inner(cfg, d, d)
    bound = 2.0 * _loglike_bound(orc, cfg, d, th[idx]) + 1e-9 * np.maximum(np.abs(L_or), sigma)
    err = np.abs(L[idx] - L_or)
    assert np.all(err <= bound), float((err / bound).max())


def test_precision_switch(torch_dev, pes):
    torch = torch_dev
    cfg = _cfg("cfg0")
    ctx = pes.Context(cfg)
    with pytest.raises(pes.PesError):
        ctx.set_precision(16)
    ctx.set_precision(32)
    ctx.set_precision(64)
    ctx.close()
