"""GPU path (libpes through its C-ABI) against the CPU oracle, element by
element on the same seeded inputs.

Tolerance rule for log L: |L_gpu - L_oracle| <= 1e-9 max(|L_oracle|, <d|d>/2).
Responses: |h_gpu - h_oracle| <= 1e-9 |h_oracle| + 1e-12 max|h_oracle| per channel.
"""
import math
import os

import numpy as np
import pytest

from paper_2602_12011_amd import workloads as W

pytestmark = pytest.mark.gpu

RTOL_L = 1e-9


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.fixture(scope="module")
def pes():
    from paper_2602_12011_amd import pes as P
    return P


def _cfg(name, n_bins=None, modes=None, dets=None):
    c = W.config(name, n_bins=n_bins)
    if modes is not None:
        c["modes"] = modes
    if dets is not None:
        c["detectors"] = dets
    return c


def _check_loglike(orc, cfg, d, L_gpu, th, what):
    L_or = orc.loglike(cfg, d, th)
    sigma = 0.5 * orc.inner(cfg, d, d)
    both_inf = np.isneginf(L_or) & np.isneginf(L_gpu)
    err = np.abs(np.where(both_inf, 0.0, L_gpu) - np.where(both_inf, 0.0, L_or))
    bound = RTOL_L * np.maximum(np.abs(np.where(both_inf, 0.0, L_or)), sigma)
    worst = np.argmax(err / bound)
    assert np.all(err <= bound), (
        f"{what}: walker {worst} theta={th[worst].tolist()} L_gpu={L_gpu[worst]!r} "
        f"L_or={L_or[worst]!r} err/bound={err[worst] / bound[worst]:.3g}")
    return np.max(err / bound)


def _run_loglike(torch, pes, cfg, d_np, th):
    ctx = pes.Context(cfg)
    d = torch.from_numpy(np.ascontiguousarray(d_np)).to("cuda")
    ctx.set_data(d)
    L = ctx.loglike(torch.from_numpy(th).to("cuda"))
    torch.cuda.synchronize()
    out = L.cpu().numpy()
    ctx.close()
    return out


CASES = {
    # name: (config, n_walkers, flat prior)
    "cfg0_full": (lambda: _cfg("cfg0"), 1000, True),
    "hm_ragged": (lambda: _cfg("cfg1", n_bins=20000 + 37), 48, False),
    "net_ragged": (lambda: _cfg("cfg2", n_bins=9000 + 5), 24, False),
    "tdi15_hm": (lambda: _cfg("cfg1", n_bins=4096 + 255,
                              dets=[dict(W.LISA, tdi_gen=15)]), 16, False),
    "taiji_only": (lambda: _cfg("cfg1", n_bins=3000, dets=[W.TAIJI]), 16, False),
    "tianqin_only": (lambda: _cfg("cfg1", n_bins=3000, dets=[W.TIANQIN]), 16, False),
}


@pytest.mark.parametrize("case", list(CASES))
def test_loglike_matches_oracle(orc, torch_dev, pes, case):
    mk, B, flat = CASES[case]
    cfg = mk()
    print(f"[parity] {case}: n_bins={cfg['n_bins']} dets={len(cfg['detectors'])} B={B}", flush=True)
    d = orc.response(cfg, W.THETA0)
    th = W.draw_walkers(B, stream=11, flat=flat)
    L = _run_loglike(torch_dev, pes, cfg, d, th)
    _check_loglike(orc, cfg, d, L, th, case)


@pytest.mark.parametrize("case", ["cfg0_full", "hm_ragged", "net_ragged", "tdi15_hm", "tianqin_only"])
def test_response_matches_oracle(orc, torch_dev, pes, case):
    """A/E/T element by element against the long-double oracle.  The T channel
    cancels as (f L)^3 relative to A and E at low frequency, so its tolerance
    also admits 1e-11 of the A/E magnitude at the same bin."""
    cfg = CASES[case][0]()
    th = np.vstack([W.THETA0, W.draw_walkers(3, stream=21, flat=CASES[case][2])])
    ctx = pes.Context(cfg)
    out = ctx.response(torch_dev.from_numpy(th).to("cuda"))
    torch_dev.cuda.synchronize()
    h_gpu = out.cpu().numpy()
    h_gpu = h_gpu[..., 0] + 1j * h_gpu[..., 1]
    ctx.close()
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


def test_edge_cases(orc, torch_dev, pes):
    cfg = _cfg("cfg1", n_bins=5000, modes=W.MODES_HM)
    d = orc.response(cfg, W.THETA0)
    th = W.draw_walkers(10, stream=31)
    th[0] = W.THETA0                        # the injection: log L ~ 0
    th[1, 1] = 1.0                          # equal masses: odd-m modes vanish
    th[2, 0] = 1e9                          # cutoff below the grid: h = 0
    th[3, 1] = 1.5                          # q > 1: unphysical
    th[4, 2] = 1.0                          # |chi| = 1: unphysical
    th[5, 0] = np.nan                       # non-finite
    th[6, 4] = -1.0                         # D_L < 0
    th[7, 0] = 1e5                          # lightest prior mass
    th[8, 3] = -0.9
    L = _run_loglike(torch_dev, pes, cfg, d, th)
    assert np.all(np.isneginf(L[3:7]))
    _check_loglike(orc, cfg, d, L, th, "edges")
    sigma = 0.5 * orc.inner(cfg, d, d)
    assert abs(L[0]) <= 1e-9 * sigma
    assert L[2] == pytest.approx(-sigma, rel=1e-12)


def test_small_batches_and_empty(orc, torch_dev, pes):
    torch = torch_dev
    cfg = _cfg("cfg0")
    d = orc.response(cfg, W.THETA0)
    ctx = pes.Context(cfg)
    ctx.set_data(torch.from_numpy(d).to("cuda"))
    empty = ctx.loglike(torch.zeros((0, 11), dtype=torch.float64, device="cuda"))
    assert empty.numel() == 0
    for B in (1, 2, 17):
        th = W.draw_walkers(B, stream=40 + B, flat=True)
        L = ctx.loglike(torch.from_numpy(th).to("cuda")).cpu().numpy()
        _check_loglike(orc, cfg, d, L, th, f"B={B}")
    ctx.close()


def test_bitwise_repeatable(orc, torch_dev, pes):
    torch = torch_dev
    cfg = _cfg("cfg2", n_bins=6000)
    d = orc.response(cfg, W.THETA0)
    ctx = pes.Context(cfg)
    ctx.set_data(torch.from_numpy(d).to("cuda"))
    th = torch.from_numpy(W.draw_walkers(300, stream=50)).to("cuda")
    a = ctx.loglike(th).cpu().numpy()
    b = ctx.loglike(th).cpu().numpy()
    perm = torch.randperm(300, generator=torch.Generator().manual_seed(1)).to("cuda")
    c = ctx.loglike(th[perm].contiguous()).cpu().numpy()
    ctx.close()
    assert np.array_equal(a, b)
    assert np.array_equal(a[perm.cpu().numpy()], c)   # independent of batch order


def test_gpu_injection_data_gives_zero_at_theta0(orc, torch_dev, pes):
    """Data made by the GPU response itself: log L(theta0) = 0 to the rounding floor."""
    torch = torch_dev
    cfg = _cfg("cfg1", n_bins=1 << 16)
    ctx = pes.Context(cfg)
    th0 = torch.from_numpy(W.THETA0[None, :].copy()).to("cuda")
    h = ctx.response(th0)[0]
    ctx.set_data(h)
    L = ctx.loglike(th0).cpu().numpy()
    ctx.close()
    sigma = 0.5 * orc.inner(cfg, orc.response(cfg, W.THETA0), orc.response(cfg, W.THETA0))
    assert abs(L[0]) <= 1e-10 * sigma


@pytest.mark.parametrize("name", ["cfg1", "cfg2"])
def test_full_size_sampled(orc, torch_dev, pes, name):
    """The benchmark's launch (all walkers of the workload, 2^20 bins) checked
    on a sample of walkers that the oracle evaluates one by one: 64 walkers at
    evenly spaced ranks of the mass order (the order in which the plan groups
    them, lightest = most tiles first), including both ends.  Run at the
    default tuning and at 24 walkers per item, whose last group is partial
    (4096 = 170 x 24 + 16, 16384 = 682 x 24 + 16), two bins per lane."""
    torch = torch_dev
    cfg = _cfg(name)
    B = cfg["walkers"]
    print(f"[parity] full-size {name}: B={B} n_bins={cfg['n_bins']}", flush=True)
    d = orc.response(cfg, W.THETA0)
    th = W.draw_walkers(B, stream=1)
    ctx = pes.Context(cfg)
    ctx.set_data(torch.from_numpy(d).to("cuda"))
    tht = torch.from_numpy(th).to("cuda")
    L = ctx.loglike(tht).cpu().numpy()
    ctx.set_tuning(2, 24, 0)
    L24 = ctx.loglike(tht).cpu().numpy()
    ctx.close()
    assert np.all(np.isfinite(L)) and np.all(L <= 0)
    order = np.argsort(th[:, 0], kind="stable")
    idx = np.unique(order[np.linspace(0, B - 1, 64).round().astype(int)])
    _check_loglike(orc, cfg, d, L[idx], th[idx], f"{name} sampled")
    _check_loglike(orc, cfg, d, L24[idx], th[idx], f"{name} sampled, 24 walkers per item")


@pytest.mark.parametrize("bpl", [1, 2])
def test_every_tuning_matches_oracle(orc, torch_dev, pes, bpl):
    """Results do not depend on the kernel tuning: every (bins per lane,
    walkers per item, blocks per CU) matches the oracle, and for a fixed tile
    size the walker grouping does not change a single bit."""
    torch = torch_dev
    cfg = _cfg("cfg2", n_bins=7000 + 3)
    d = orc.response(cfg, W.THETA0)
    th = W.draw_walkers(100, stream=60)
    ctx = pes.Context(cfg)
    ctx.set_data(torch.from_numpy(d).to("cuda"))
    tht = torch.from_numpy(th).to("cuda")
    ref = None
    for wg, bpc in ((1, 0), (7, 1), (16, 0), (64, 2)):
        ctx.set_tuning(bpl, wg, bpc)
        L = ctx.loglike(tht).cpu().numpy()
        _check_loglike(orc, cfg, d, L, th, f"bpl={bpl} wg={wg} bpc={bpc}")
        if ref is None:
            ref = L
        assert np.array_equal(L, ref)
    ms, tun = ctx.autotune(tht)
    assert ms > 0 and tun["bins_per_lane"] in (1, 2)
    L = ctx.loglike(tht).cpu().numpy()
    _check_loglike(orc, cfg, d, L, th, f"autotuned {tun}")
    ctx.close()


def test_plain_grid_schedule_is_bitwise_the_queue(orc, torch_dev, pes):
    """The plain-grid schedule (every tile, batch order) and the persistent
    queue (active tiles, sorted walkers) give the same bits; one unphysical
    walker (q > 1) stays at -inf under both."""
    torch = torch_dev
    cfg = _cfg("cfg2", n_bins=7000 + 3)
    d = orc.response(cfg, W.THETA0)
    th = W.draw_walkers(100, stream=61)
    th[7, 1] = 1.5
    ctx = pes.Context(cfg)
    ctx.set_data(torch.from_numpy(d).to("cuda"))
    tht = torch.from_numpy(th).to("cuda")
    assert pes.lib().pes_set_schedule(ctx.h, 7) == -1     # PES_EINVAL
    for bpl, wg in ((1, 1), (1, 16), (2, 7), (2, 64)):
        ctx.set_tuning(bpl, wg, 0)
        ctx.set_schedule("queue")
        Lq = ctx.loglike(tht).cpu().numpy()
        ctx.set_schedule("grid")
        Lg = ctx.loglike(tht).cpu().numpy()
        assert np.array_equal(Lq, Lg), (bpl, wg)
        assert np.isneginf(Lg[7])
    _check_loglike(orc, cfg, d, Lg, th, "plain grid")
    ctx.close()


def test_work_item_bound(torch_dev, pes):
    """The (walker group, tile) plan is int32: a batch whose item count would
    exceed it is refused with PES_ESHAPE before any work is queued, under both
    schedules; a larger walkers-per-item tuning brings it back within range."""
    torch = torch_dev
    cfg = _cfg("cfg1", n_bins=1 << 22)          # 16384 tiles of 256 bins
    cfg["df"] = cfg["df"] / 4                   # up to 33 mHz: inside the sinc fits' range
    ctx = pes.Context(cfg)
    ctx.set_data(torch.zeros((1, 3, cfg["n_bins"], 2), dtype=torch.float64, device="cuda"))
    B = (1 << 17) + 1                           # 131073 groups of one walker
    th = torch.from_numpy(W.draw_walkers(B, stream=95)).to("cuda")
    out = torch.empty(B, dtype=torch.float64, device="cuda")
    for sched in ("queue", "grid"):
        ctx.set_schedule(sched)
        ctx.set_tuning(1, 1, 0)
        rc = pes.lib().pes_loglike(ctx.h, pes._dev_f64(th, "theta"), B, pes._dev_f64(out, "logl"), None)
        assert rc == -2, (sched, rc)
    ctx.close()
