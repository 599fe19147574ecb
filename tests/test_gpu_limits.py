"""The largest sizes the boundary accepts, through the C-ABI.  Batches, on a
short ragged grid (259 bins of the 2^20-bin LISA grid, five modes):
pes_loglike at B = 2^24 walkers and pes_grad / pes_fisher at B = 65535, their
stated limits.  Every walker is checked for what holds at any size (finite,
log L <= 0 on noise-free data), and walkers at the ends and in the middle of
the batch against the oracle at the FP64 bars: log L to 1e-9 max(|L|,
<d|d>/2), gradients to 1e-6 of their scale in prior-width units, Fisher
entries to 1e-6 of sqrt(F_ii F_jj).  One walker beyond each limit is refused
(PES_EINVAL).  Grid: log L on 2^26 bins (df = 1e-9 Hz from 1e-4 Hz, five
modes, LISA; the long-sinc kernels) against the sum over its parts and, at the
grid's top, the oracle; 2^26 + 1 bins refused by pes_create."""
import numpy as np
import pytest

from paper_2602_12011_amd import workloads as W

pytestmark = pytest.mark.gpu

MAX_LOGLIKE = 1 << 24
MAX_DERIV = 65535


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.fixture(scope="module")
def pes():
    from paper_2602_12011_amd import pes as P
    return P


def _cfg():
    return W.config("cfg1", n_bins=256 + 3)


def _sample(B, rng):
    """Walkers at both ends, in the middle and at random places of the batch."""
    return np.unique(np.concatenate([[0, 1, B // 2, B - 2, B - 1], rng.integers(0, B, 3)]))


def test_loglike_at_the_batch_limit(orc, torch_dev, pes):
    torch = torch_dev
    cfg = _cfg()
    B = MAX_LOGLIKE
    print(f"[limits] loglike B={B} n_bins={cfg['n_bins']}", flush=True)
    d = orc.response(cfg, W.THETA0)
    th = W.draw_walkers(B, stream=61)
    ctx = pes.Context(cfg)
    ctx.set_data(torch.from_numpy(np.ascontiguousarray(d)).to("cuda"))
    tht = torch.from_numpy(th).to("cuda")
    L = ctx.loglike(tht).cpu().numpy()
    del tht
    with pytest.raises(pes.PesError):
        ctx.loglike(torch.zeros((B + 1, 11), dtype=torch.float64, device="cuda"))
    ctx.close()
    sigma = 0.5 * orc.inner(cfg, d, d)
    assert np.all(np.isfinite(L)), int(np.sum(~np.isfinite(L)))
    assert np.all(L <= 1e-9 * sigma)
    idx = _sample(B, np.random.default_rng(7))
    L_or = orc.loglike(cfg, d, th[idx])
    err = np.abs(L[idx] - L_or)
    assert np.all(err <= 1e-9 * np.maximum(np.abs(L_or), sigma)), (idx, err)
    print(f"[limits] loglike: {idx.size} sampled walkers within the bar", flush=True)


@pytest.mark.parametrize("method", ["adjoint", "forward"])
def test_grad_at_the_batch_limit(orc, torch_dev, pes, method):
    torch = torch_dev
    cfg = _cfg()
    B = MAX_DERIV
    print(f"[limits] grad {method} B={B} n_bins={cfg['n_bins']}", flush=True)
    d = orc.response(cfg, W.THETA0)
    th = W.draw_walkers(B, stream=62)
    ctx = pes.Context(cfg)
    ctx.set_grad_method(method)
    ctx.set_data(torch.from_numpy(np.ascontiguousarray(d)).to("cuda"))
    L, g = ctx.grad(torch.from_numpy(th).to("cuda"))
    L, g = L.cpu().numpy(), g.cpu().numpy()
    with pytest.raises(pes.PesError):
        ctx.grad(torch.zeros((B + 1, 11), dtype=torch.float64, device="cuda"))
    ctx.close()
    assert np.all(np.isfinite(L)) and np.all(np.isfinite(g))
    idx = _sample(B, np.random.default_rng(8))
    L_or, g_or = orc.grad(cfg, d, th[idx])
    sigma = 0.5 * orc.inner(cfg, d, d)
    assert np.all(np.abs(L[idx] - L_or) <= 1e-9 * np.maximum(np.abs(L_or), sigma))
    s = W.prior_widths()
    for r, b in enumerate(idx):
        scale = np.abs(g_or[r] * s).max()
        err = np.abs(g[b] - g_or[r]) * s
        assert np.all(err <= 1e-6 * scale), (method, b, (err / scale).max())


def test_fisher_at_the_batch_limit(orc, torch_dev, pes):
    torch = torch_dev
    cfg = _cfg()
    B = MAX_DERIV
    print(f"[limits] fisher B={B} n_bins={cfg['n_bins']}", flush=True)
    th = W.draw_walkers(B, stream=63)
    ctx = pes.Context(cfg)
    F = ctx.fisher(torch.from_numpy(th).to("cuda")).cpu().numpy()
    with pytest.raises(pes.PesError):
        ctx.fisher(torch.zeros((B + 1, 11), dtype=torch.float64, device="cuda"))
    ctx.close()
    assert np.all(np.isfinite(F))
    idx = _sample(B, np.random.default_rng(9))
    F_or = orc.fisher(cfg, th[idx])
    for r, b in enumerate(idx):
        dg = np.sqrt(np.outer(np.diag(F_or[r]), np.diag(F_or[r])))
        err = np.abs(F[b] - F_or[r]) / dg
        assert np.all(err <= 1e-6), (b, err.max())


def test_loglike_at_the_bin_limit(orc, torch_dev, pes):
    """2^26 bins (the limit), five modes, zero data (log L = -<h|h>/2): a bin
    sum, so the full grid's log L equals the sum over 16 contexts on its
    consecutive sixteenths (2^22 bins each) to rounding; its first and its
    last 4099 bins against the oracle."""
    torch = torch_dev
    N = 1 << 26
    base = dict(W.config("cfg1"), df=1e-9)
    cfg = dict(base, n_bins=N, f0=1e-4)
    print(f"[limits] loglike n_bins={N}", flush=True)
    th = np.vstack([W.THETA0, W.draw_walkers(2, stream=64)])
    th[1, 0], th[2, 0] = 1e5, 5e6                  # a light walker spans most of the grid
    tht = torch.from_numpy(th).to("cuda")

    def run(c):
        ctx = pes.Context(c)
        ctx.set_data(torch.zeros((1, 3, c["n_bins"], 2), dtype=torch.float64, device="cuda"))
        L = ctx.loglike(tht).cpu().numpy()
        ctx.close()
        return L

    L_full = run(cfg)
    M = N // 16
    L_parts = sum(run(dict(base, n_bins=M, f0=cfg["f0"] + i * M * cfg["df"])) for i in range(16))
    assert np.all(np.isfinite(L_full)) and np.all(L_full < 0)
    assert np.allclose(L_full, L_parts, rtol=1e-10, atol=0), (L_full, L_parts)
    for k0 in (0, N - 4099):          # where every walker has signal, and the grid's top
        sub = dict(base, n_bins=4099, f0=cfg["f0"] + k0 * cfg["df"])
        L_sub = run(sub)
        L_or = orc.loglike(sub, np.zeros((1, 3, 4099), dtype=complex), th)
        assert np.all(np.abs(L_sub - L_or) <= 1e-9 * np.abs(L_or)), (k0, L_sub, L_or)
    with pytest.raises(pes.PesError):
        pes.Context(dict(cfg, n_bins=N + 1))
    print(f"[limits] bins: full grid against its 16 parts {float(np.abs(L_full / L_parts - 1).max()):.1e}",
          flush=True)
