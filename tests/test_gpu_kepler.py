"""Exact Keplerian heliocentric orbits (detector option orbit = 'kepler')
through the C-ABI against the oracle's exact Kepler ellipses: log L per walker
to 1e-9 max(|L|, <d|d>/2) and A/E/T element by element to 1e-9 |h| + 1e-12
max|h| (T also 1e-11 of the A/E magnitude), as for the first-order orbit, on
LISA alone, on the three-detector network (TianQin stays geocentric), on the
paper's 32703-bin grid (long sinc fits) and with TDI 1.5; both bin-per-lane
kernel variants.  Gradients (forward mode, whichever method is set) and Fisher
matrices against the oracle's dual numbers on the same orbits, at the
tolerances of the first-order orbit's derivative tests.  Single precision and
the stage probes on these orbits are tested with the other FP32 cases and
stage tests."""
import numpy as np
import pytest

from paper_2602_12011_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.fixture(scope="module")
def pes():
    from paper_2602_12011_amd import pes as P
    return P


def _kep(det):
    return det if det["kind"] == "tianqin" else dict(det, orbit="kepler")


def _cfg(name, n_bins=None, tdi15=False):
    c = W.config(name, n_bins=n_bins)
    dets = [_kep(d) for d in c["detectors"]]
    if tdi15:
        dets = [dict(d, tdi_gen=15) for d in dets]
    c["detectors"] = dets
    return c


CASES = {
    "lisa_hm": (lambda: _cfg("cfg1", n_bins=20000 + 37), W.THETA0, 40),
    "network": (lambda: _cfg("cfg2", n_bins=9000 + 5), W.THETA0, 24),
    "pe_grid": (lambda: _cfg("pehm"), W.THETA_PE, 16),
    "tdi15": (lambda: _cfg("cfg1", n_bins=4096 + 255, tdi15=True), W.THETA0, 16),
}


@pytest.mark.parametrize("case", list(CASES))
def test_kepler_loglike_matches_oracle(orc, torch_dev, pes, case):
    torch = torch_dev
    mk, inj, B = CASES[case]
    cfg = mk()
    d = orc.response(cfg, inj)
    th = np.vstack([inj, W.draw_walkers(B - 1, stream=17)])
    if case == "pe_grid":
        th[1:, 10] += W.THETA_PE[10] - W.THETA0[10]
        th[1, 0] = 1.0e5                       # a light walker reaches the long-sinc bins
    print(f"[kepler] loglike {case}: n_bins={cfg['n_bins']} dets={len(cfg['detectors'])} B={B}", flush=True)
    ctx = pes.Context(cfg)
    ctx.set_data(torch.from_numpy(np.ascontiguousarray(d)).to("cuda"))
    tht = torch.from_numpy(th).to("cuda")
    Ls = []
    for bpl, wg in ((1, 16), (2, 5)):
        ctx.set_tuning(bpl, wg, 0)
        Ls.append(ctx.loglike(tht).cpu().numpy())
    Ln = ctx.loglike_noalloc(tht).cpu().numpy()
    ctx.close()
    assert np.array_equal(Ln, Ls[1])
    L_or = orc.loglike(cfg, d, th)
    sigma = 0.5 * orc.inner(cfg, d, d)
    for L in Ls:
        err = np.abs(L - L_or)
        bound = 1e-9 * np.maximum(np.abs(L_or), sigma)
        w = int(np.argmax(err / bound))
        assert np.all(err <= bound), (case, w, L[w], L_or[w], err[w] / bound[w])
    print(f"[kepler] loglike {case}: worst err / bound {float((np.abs(Ls[0] - L_or) / (1e-9 * np.maximum(np.abs(L_or), sigma))).max()):.3f}",
          flush=True)


@pytest.mark.parametrize("case", list(CASES))
def test_kepler_response_matches_oracle(orc, torch_dev, pes, case):
    torch = torch_dev
    mk, inj, _ = CASES[case]
    cfg = mk()
    th = np.vstack([inj, W.draw_walkers(2, stream=23)])
    if case == "pe_grid":
        th[1:, 10] += W.THETA_PE[10] - W.THETA0[10]
        th[1, 0] = 1.0e5
    ctx = pes.Context(cfg)
    out = ctx.response(torch.from_numpy(th).to("cuda")).cpu().numpy()
    ctx.close()
    h_gpu = out[..., 0] + 1j * out[..., 1]
    for b in range(th.shape[0]):
        h_or = orc.response(cfg, th[b], prec=1)
        for det in range(h_or.shape[0]):
            ae = np.sqrt(np.abs(h_or[det, 0]) ** 2 + np.abs(h_or[det, 1]) ** 2)
            for c in range(3):
                ref = h_or[det, c]
                tol = 1e-9 * np.abs(ref) + 1e-12 * np.abs(ref).max()
                if c == 2:
                    tol = tol + 1e-11 * ae
                err = np.abs(h_gpu[b, det, c] - ref)
                assert np.all(err <= tol), (case, b, det, c, float((err / tol).max()))


def test_kepler_differs_from_first_order(orc, torch_dev, pes):
    """The GPU's exact-orbit response is not the first-order one: the two
    differ by the oracle's own difference (order e^2 AU / L)."""
    torch = torch_dev
    kep = _cfg("cfg1", n_bins=5000)
    first = W.config("cfg1", n_bins=5000)
    th = torch.from_numpy(W.THETA0[None, :].copy()).to("cuda")
    outs = []
    for cfg in (kep, first):
        ctx = pes.Context(cfg)
        o = ctx.response(th).cpu().numpy()
        outs.append(o[..., 0] + 1j * o[..., 1])
        ctx.close()
    diff_gpu = outs[0][0] - outs[1][0]
    diff_or = orc.response(kep, W.THETA0, prec=1) - orc.response(first, W.THETA0, prec=1)
    scale = np.abs(outs[1][0]).max()
    assert np.abs(diff_or).max() > 1e-4 * scale
    assert np.abs(diff_gpu - diff_or).max() <= 1e-8 * scale


def test_kepler_full_size_sampled(orc, torch_dev, pes):
    """The benchmark's Kepler launch (4096 walkers, 2^20 bins, five modes) on a
    sample of walkers the oracle evaluates one by one: 16 at evenly spaced
    ranks of the mass order, both ends included; autotuned and at 24 walkers
    per item with two bins per lane (a partial last group)."""
    torch = torch_dev
    cfg = _cfg("cfg1")
    B = cfg["walkers"]
    print(f"[kepler] full size: B={B} n_bins={cfg['n_bins']}", flush=True)
    d = orc.response(cfg, W.THETA0)
    th = W.draw_walkers(B, stream=1)
    ctx = pes.Context(cfg)
    ctx.set_data(torch.from_numpy(np.ascontiguousarray(d)).to("cuda"))
    tht = torch.from_numpy(th).to("cuda")
    ctx.autotune(tht)
    L = ctx.loglike(tht).cpu().numpy()
    ctx.set_tuning(2, 24, 0)
    L24 = ctx.loglike(tht).cpu().numpy()
    ctx.close()
    assert np.all(np.isfinite(L)) and np.all(L <= 0)
    order = np.argsort(th[:, 0], kind="stable")
    idx = np.unique(order[np.linspace(0, B - 1, 16).round().astype(int)])
    L_or = orc.loglike(cfg, d, th[idx])
    sigma = 0.5 * orc.inner(cfg, d, d)
    for got in (L[idx], L24[idx]):
        err = np.abs(got - L_or)
        assert np.all(err <= 1e-9 * np.maximum(np.abs(L_or), sigma)), float(
            (err / (1e-9 * np.maximum(np.abs(L_or), sigma))).max())


DERIV_CASES = {
    "lisa_hm": (lambda: _cfg("cfg1", n_bins=3000 + 17), W.THETA0),
    "network": (lambda: _cfg("cfg2", n_bins=2000 + 9), W.THETA0),
    "pe_grid": (lambda: _cfg("pehm"), W.THETA_PE),
}


def _walkers(case, inj, n, stream):
    th = np.vstack([inj + 1e-5 * W.prior_widths(), W.draw_walkers(n - 1, stream=stream)])
    if case == "pe_grid":
        th[1:, 10] += W.THETA_PE[10] - W.THETA0[10]
        th[1, 0] = 1.0e5                       # a light walker reaches the long-sinc bins
    return th


@pytest.mark.parametrize("method", ["adjoint", "forward"])
@pytest.mark.parametrize("case", list(DERIV_CASES))
def test_kepler_grad_matches_oracle(orc, torch_dev, pes, case, method):
    torch = torch_dev
    mk, inj = DERIV_CASES[case]
    cfg = mk()
    d = orc.response(cfg, inj)
    th = _walkers(case, inj, 3 if case == "pe_grid" else 5, 73)
    print(f"[kepler] grad {case} {method}: n_bins={cfg['n_bins']} dets={len(cfg['detectors'])}", flush=True)
    ctx = pes.Context(cfg)
    ctx.set_grad_method(method)
    ctx.set_data(torch.from_numpy(np.ascontiguousarray(d)).to("cuda"))
    tht = torch.from_numpy(th).to("cuda")
    L, g = ctx.grad(tht)
    L, g = L.cpu().numpy(), g.cpu().numpy()
    L_ll = ctx.loglike(tht).cpu().numpy()
    ctx.close()
    L_or, g_or = orc.grad(cfg, d, th)
    sigma = 0.5 * orc.inner(cfg, d, d)
    assert np.all(np.abs(L - L_or) <= 1e-9 * np.maximum(np.abs(L_or), sigma))
    assert np.all(np.abs(L - L_ll) <= 1e-10 * np.maximum(np.abs(L_ll), sigma))
    s = W.prior_widths()
    for b in range(th.shape[0]):
        scale = np.abs(g_or[b] * s).max()
        err = np.abs(g[b] - g_or[b]) * s
        assert np.all(err <= 1e-6 * scale), (case, b, (err / scale).max())


@pytest.mark.parametrize("case", list(DERIV_CASES))
def test_kepler_fisher_matches_oracle(orc, torch_dev, pes, case):
    torch = torch_dev
    mk, inj = DERIV_CASES[case]
    cfg = mk()
    th = _walkers(case, inj, 3, 74)
    print(f"[kepler] fisher {case}: n_bins={cfg['n_bins']}", flush=True)
    ctx = pes.Context(cfg)
    F = ctx.fisher(torch.from_numpy(th).to("cuda")).cpu().numpy()
    ctx.close()
    F_or = orc.fisher(cfg, th)
    assert np.allclose(F, np.transpose(F, (0, 2, 1)), rtol=1e-12, atol=0)
    for b in range(th.shape[0]):
        dg = np.sqrt(np.outer(np.diag(F_or[b]), np.diag(F_or[b])))
        err = np.abs(F[b] - F_or[b]) / dg
        assert np.all(err <= 1e-6), (case, b, err.max(), np.unravel_index(err.argmax(), err.shape))


def test_kepler_fisher_differs_from_first_order(orc, torch_dev, pes):
    """The exact orbits change the Fisher matrix by the oracle's own amount."""
    torch = torch_dev
    kep = _cfg("cfg1", n_bins=3000)
    first = W.config("cfg1", n_bins=3000)
    th = torch.from_numpy(W.THETA0[None, :].copy()).to("cuda")
    Fs = []
    for cfg in (kep, first):
        ctx = pes.Context(cfg)
        Fs.append(ctx.fisher(th).cpu().numpy()[0])
        ctx.close()
    F_or = orc.fisher(kep, W.THETA0[None, :])[0] - orc.fisher(first, W.THETA0[None, :])[0]
    dg = np.sqrt(np.outer(np.diag(Fs[1]), np.diag(Fs[1])))
    assert np.abs(F_or / dg).max() > 1e-6
    assert np.abs((Fs[0] - Fs[1] - F_or) / dg).max() <= 2e-6


def test_kepler_refusals(pes):
    """Configurations the orbit option does not define: heliocentric detectors
    on different orbit models in one context, and a geocentric detector on
    Kepler ellipses."""
    mixed = dict(W.config("cfg2", n_bins=1000))
    mixed["detectors"] = [dict(W.LISA, orbit="kepler"), W.TAIJI, W.TIANQIN]
    with pytest.raises(pes.PesError):
        pes.Context(mixed)
    with pytest.raises(pes.PesError):
        pes.Context(dict(mixed, detectors=[dict(W.TIANQIN, orbit="kepler")]))
