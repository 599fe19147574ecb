"""Benchmark: batched FP64 log-likelihood evaluations per second on one MI355X.

Workload (one step = one pes_loglike call = the whole hot path: walker setup,
work plan, persistent response + inner-product kernel, per-walker reduction):
one LISA-like detector, modes (2,2),(2,1),(3,3),(3,2),(4,4), 2^20 frequency
bins at df = 1/yr from 1e-4 Hz, 4096 walkers drawn from the prior box with
log-uniform total mass 1e5..1e7 Msun, noise-free data injected at the
reference source (generated on the GPU by pes_response).

Prints one JSON line with the measured throughput, a roofline entry for the
dominant kernel (FP64 vector ALU bound) and the CPU oracle timed on a bounded
sample of the same workload.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2602_12011_amd import workloads as W  # noqa: E402

METRIC = "logL evals/s @2^20 bins, 5 modes (FP64); ESS/s learned vs plain proposal"
PEAK_FP64_VECTOR_TFLOPS = 78.6     # MI355X FP64 vector peak (AMD specification)

# FP64 operations (FMA counted as 2) of the kernel's formulation, counted from
# its source: per active (walker, bin, detector, mode) unit -- heliocentric or
# geocentric orbit, short or long sinc fit, fit class of the bin's wavefront --
# and per active (walker, bin, detector) for the TDI combination and the inner
# products.  Not counted: the C^2 taper (the last 10% below each cutoff) and
# the quarter-turn rotation of the sine/cosine reduction (products with 0 and
# +-1).  A wavefront of 64 consecutive bins whose largest link sinc argument
# 2 pi f L stays at or below 0.5 (class 0) evaluates the sinc and the arm
# phases with shorter fits of that range; class 1 is the full range.
FLOPS_PER_MODE_UNIT = {("helio", False, 1): 442, ("geo", False, 1): 469,
                       ("helio", True, 1): 474, ("geo", True, 1): 501,
                       ("helio", False, 0): 390, ("geo", False, 0): 417,
                       ("helio", True, 0): 390, ("geo", True, 0): 417}
# A mode with the same m as an earlier one (the first such pair per m) rides on
# that mode's unit: its amplitude, the rotated polarization factors and the
# complex products with the phase factor cost 19 flops instead of a unit.
FLOPS_PER_PAIRED_MODE = 19
FLOPS_PER_WBD_UNIT = 83
CLASS_BMAX0 = 0.5
MF_ISCO = 6.0 ** -1.5 / math.pi
MSUN_S = 4.925490947641267e-6


def mode_bin_counts(cfg, theta):
    """Active bins per (walker, mode) -- bins k < n below the mode's cutoff --
    and, per walker, the largest of them."""
    N, f0, df = cfg["n_bins"], cfg["f0"], cfg["df"]
    M = theta[:, 0] * MSUN_S
    ns = []
    for (l, m) in cfg["modes"]:
        fcut = 0.5 * m * MF_ISCO / M
        ns.append(np.clip(np.ceil((fcut - f0) / df), 0, N).astype(np.int64))
    ns = np.stack(ns, axis=1)
    return ns, ns.max(axis=1)


def active_units(cfg, theta):
    """(mode units, walker-bin units) per detector that one pes_loglike evaluates."""
    ns, nmax = mode_bin_counts(cfg, theta)
    return float(ns.sum()), float(nmax.sum())


def paired_modes(modes):
    """Indices of the modes evaluated on an earlier mode's unit (same m)."""
    out, seen = set(), set()
    for j, (l, m) in enumerate(modes):
        if m in seen:
            continue
        seen.add(m)
        for i in range(j + 1, len(modes)):
            if modes[i][1] == m:
                out.add(i)
                break
    return out


def bin_classes(cfg, det):
    """Fit class of every bin: that of its aligned 64-bin wavefront."""
    N = cfg["n_bins"]
    L = det["arm_m"] / 299792458.0
    k = np.arange(((N + 63) // 64) * 64)
    f = cfg["f0"] + np.minimum(k, N - 1) * cfg["df"]
    bmax = (2 * math.pi * L * f).reshape(-1, 64).max(axis=1)
    cls = np.where(bmax <= CLASS_BMAX0, 0, 1)
    return np.repeat(cls, 64)[:N]


def algorithmic_flops(cfg, theta):
    ns, nmax = mode_bin_counts(cfg, theta)
    n_mode, n_wb = float(ns.sum()), float(nmax.sum())
    f_max = cfg["f0"] + (cfg["n_bins"] - 1) * cfg["df"]
    total = 0.0
    for d in cfg["detectors"]:
        L = d["arm_m"] / 299792458.0
        long_sinc = (2 * math.pi * f_max * L) ** 2 > 4.9
        orbit = "geo" if d["kind"] == "tianqin" else "helio"
        cls = bin_classes(cfg, d)
        paired = sorted(paired_modes(cfg["modes"]))
        units = [j for j in range(ns.shape[1]) if j not in paired]
        for c in range(2):
            cum = np.concatenate([[0], np.cumsum(cls == c)])
            total += FLOPS_PER_MODE_UNIT[(orbit, long_sinc, c)] * float(cum[ns[:, units]].sum())
        total += FLOPS_PER_PAIRED_MODE * float(ns[:, paired].sum())
        total += FLOPS_PER_WBD_UNIT * n_wb
    nd = len(cfg["detectors"])
    return total, n_mode * nd, n_wb * nd


KERNEL_SOURCES = ("pes_eval.hpp", "pes_kernels.hip", "pes_math.hpp", "pes_poly.hpp",
                  "pes_layout.hpp", "pes_launch.hpp", "pes_eval32.hpp")
COUNTER_SUMMARY = os.path.join(ROOT, "profiles", "loglike_kernel_cfg1_counters.md")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2602_12011_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(tuning):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel sources with the same tuning; else None."""
    try:
        text = open(COUNTER_SUMMARY).read()
    except OSError:
        return None
    tun = f"{tuning['bins_per_lane']},{tuning['walkers_per_group']},{tuning['blocks_per_cu']}"
    vals = {}
    for line in text.splitlines():
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_sources_sha256_16") != kernel_source_hash():
        return None
    v = vals.get(f"traffic_bytes_per_launch[{tun}]")
    return float(v) if v is not None else None


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(cfg, theta, n_sample, threads, n_single=4):
    """The oracle on the host: n_sample walkers over `threads` threads (OpenMP
    over walkers), and n_single walkers on one thread."""
    import oracle
    d = oracle.response(cfg, W.THETA0)
    sample = theta[:n_sample]
    oracle.loglike(cfg, d, sample[:1], nthreads=threads)   # load + warm
    t0 = time.perf_counter()
    oracle.loglike(cfg, d, sample, nthreads=threads)
    dt = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.loglike(cfg, d, theta[:n_single], nthreads=1)
    dt1 = time.perf_counter() - t0
    return dict(value=n_sample / dt, unit="logL evals/s", cores=threads, kind="oracle",
                sample=f"{n_sample} of the {len(theta)} walkers, full {cfg['n_bins']}-bin grid, "
                       f"5 modes, {dt:.1f} s wall",
                one_thread=dict(value=n_single / dt1, sample=f"{n_single} walkers, {dt1:.1f} s wall"),
                cpu_model=_cpu_model(), host_cpus=os.cpu_count())


def _time_ms(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def derivative_leg(torch, pes, reps):
    """Gradients (reverse and forward mode) at 1024 walkers and Fisher matrices
    at 256 points on cfg1's signal and grid (2^20 bins, 5 modes)."""
    cfg = W.config("cfg3")
    dev = torch.device("cuda:0")
    ctx = pes.Context(cfg)
    th0 = torch.from_numpy(W.THETA0[None, :].copy()).to(dev)
    ctx.set_data(ctx.response(th0)[0].clone())
    th = torch.from_numpy(W.draw_walkers(cfg["walkers"], stream=3)).to(dev)
    thf = th[:cfg["fisher_points"]].contiguous()
    out = {}
    t_ll = _time_ms(torch, lambda: ctx.loglike(th), reps)
    ctx.set_grad_method("adjoint")
    t_adj = _time_ms(torch, lambda: ctx.grad(th), reps)
    ctx.set_grad_method("forward")
    t_fwd = _time_ms(torch, lambda: ctx.grad(th), max(1, reps // 2))
    t_fis = _time_ms(torch, lambda: ctx.fisher(thf), max(1, reps // 2))
    ctx.close()
    B, Bf = cfg["walkers"], cfg["fisher_points"]
    out = dict(workload="LISA-like, 5 modes, 2^20 bins; gradients at 1024 walkers, Fisher at 256",
               loglike_ms=round(t_ll, 3), grad_adjoint_ms=round(t_adj, 3), grad_forward_ms=round(t_fwd, 3),
               fisher_ms=round(t_fis, 3), grad_evals_per_s=round(B / (t_adj * 1e-3), 1),
               grad_over_loglike=round(t_adj / t_ll, 3), adjoint_speedup_over_forward=round(t_fwd / t_adj, 2),
               fisher_per_s=round(Bf / (t_fis * 1e-3), 1))
    return out


def graph_leg(torch, pes, steps):
    """Sampler steps/s, eager steps against one captured-graph replay per
    step: at the small workload (1000 walkers, 4096 bins, (2,2)), and at a
    batch small enough for the launches to dominate (64 walkers, the first
    512 of those bins)."""
    def one(B, n_bins):
        cfg = W.config("cfg0", n_bins=n_bins)
        dev = torch.device("cuda:0")
        ctx = pes.Context(cfg)
        th0 = torch.from_numpy(W.THETA0[None, :].copy()).to(dev)
        ctx.set_data(ctx.response(th0)[0].clone())
        prior = _prior_spec()
        rng = np.random.default_rng(11)
        start = torch.from_numpy(W.THETA0 + 1e-6 * W.prior_widths() * rng.normal(size=(B, 11))).to(dev)
        a = pes.Sampler(ctx, prior, B, 5)
        b = pes.Sampler(ctx, prior, B, 5)
        a.set_state(start)
        b.set_state(start)
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            b.capture(s)
            t_graph = _time_ms(torch, lambda: b.launch(1, s), steps)
        t_eager = _time_ms(torch, lambda: a.step(1), steps)
        a.close()
        b.close()
        ctx.close()
        return t_eager, t_graph
    te, tg = one(1000, None)
    te_s, tg_s = one(64, 512)
    return dict(workload="1000 walkers, 4096 bins, (2,2) mode, LISA-like", eager_ms_per_step=round(te, 4),
                graph_ms_per_step=round(tg, 4), graph_speedup=round(te / tg, 3),
                small=dict(workload="64 walkers, 512 bins, (2,2) mode, LISA-like", eager_ms_per_step=round(te_s, 4),
                           graph_ms_per_step=round(tg_s, 4), graph_speedup=round(te_s / tg_s, 3)))


def schedule_utilisation(cfg, theta, tile, grid):
    """Share of the walker-bins a schedule processes that lie below the
    walker's highest mode cutoff, and the share of its mode slots (walker-bins
    x modes) that are active."""
    ns, nmax = mode_bin_counts(cfg, theta)
    N = cfg["n_bins"]
    if grid:
        processed = len(theta) * ((N + tile - 1) // tile) * tile
    else:   # the kernel's active tiles cover one bin beyond the highest cutoff
        nact = np.minimum(nmax + 1, N)
        processed = float((((nact + tile - 1) // tile) * tile).sum())
    return float(nmax.sum()) / processed, float(ns.sum()) / (processed * len(cfg["modes"]))


def config2_leg(torch, pes, reps):
    """Three detectors, 16384 walkers, 2^20 bins, 5 modes: the persistent
    queue against a plain grid, the default tuning against the autotuned
    one, eager calls against one captured-graph replay."""
    cfg = W.config("cfg2")
    B = cfg["walkers"]
    dev = torch.device("cuda:0")
    theta_np = W.draw_walkers(B, stream=2)
    ctx = pes.Context(cfg)
    ctx.reserve(B)
    th0 = torch.from_numpy(W.THETA0[None, :].copy()).to(dev)
    ctx.set_data(ctx.response(th0)[0].clone())
    theta = torch.from_numpy(theta_np).to(dev)
    out = torch.empty(B, dtype=torch.float64, device=dev)

    def run():
        ctx.loglike(theta, out)

    res = dict(workload="LISA+Taiji+TianQin, 5 modes, 2^20 bins, 16384 walkers")
    tun0 = ctx.get_tuning()
    t_default = _time_ms(torch, run, reps)
    _, tun = ctx.autotune(theta)
    t_queue = _time_ms(torch, run, reps)
    L_queue = out.cpu().numpy()
    ctx.set_schedule("grid")
    t_grid = _time_ms(torch, run, reps)
    L_grid = out.cpu().numpy()
    ctx.set_schedule("queue")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        run()
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run()
    t_graph = _time_ms(torch, g.replay, reps)
    L_graph = out.cpu().numpy()
    ctx.close()
    tile = 256 * tun["bins_per_lane"]
    uq = schedule_utilisation(cfg, theta_np, tile, False)
    ug = schedule_utilisation(cfg, theta_np, tile, True)
    res.update(
        default_tuning=tun0, autotuned_tuning=tun,
        queue_default_tuning_ms=round(t_default, 2), queue_autotuned_ms=round(t_queue, 2),
        grid_autotuned_ms=round(t_grid, 2), queue_graph_replay_ms=round(t_graph, 2),
        evals_per_s=round(B / (t_queue * 1e-3), 1),
        queue_speedup_over_grid=round(t_grid / t_queue, 3),
        autotune_speedup=round(t_default / t_queue, 3),
        graph_speedup=round(t_queue / t_graph, 4),
        queue_walker_bin_utilisation=round(uq[0], 4), queue_mode_slot_utilisation=round(uq[1], 4),
        grid_walker_bin_utilisation=round(ug[0], 4), grid_mode_slot_utilisation=round(ug[1], 4),
        grid_bitwise_equal=bool(np.array_equal(L_queue, L_grid)),
        graph_bitwise_equal=bool(np.array_equal(L_queue, L_graph)))
    return res


def _pe_walkers(n, stream):
    """Prior draws with t_c moved to the paper's injection epoch."""
    th = W.draw_walkers(n, stream=stream)
    th[:, 10] += W.THETA_PE[10] - W.THETA0[10]
    return th


def _noisy_context(torch, pes, cfg, seed, reserve):
    """Context with data = response(THETA_PE) + one Gaussian noise realisation."""
    dev = torch.device("cuda:0")
    ctx = pes.Context(cfg)
    ctx.reserve(reserve)
    thp = torch.from_numpy(W.THETA_PE[None, :].copy()).to(dev)
    h0 = ctx.response(thp)[0].clone()
    n = ctx.noise(seed)
    return ctx, thp, h0, n


def paper_pe_leg(torch, pes, batch=1024, n_single=10, reps=5):
    """The paper's PE set-up (655360 s at 10 s, 32703 bins, its injection, its
    three scenarios) with Gaussian noise from pes_noise: SNR, log L at the
    injection against the noise's expectation, and log L evals/s one sample
    per call (the paper's protocol; eager and as a graph replay) and batched.
    Then the paper's cost-vs-bins axis: series of 10 s x 2^p samples, p =
    12..21, LISA-like with five modes, per-sample time at one sample per call
    and in batches."""
    dev = torch.device("cuda:0")
    out = dict(workload="paper's PE grid: 655360 s at 10 s, rfftfreq bins in [1e-4, 5e-2] Hz (32703), "
                        "its injection (Table tab_pe_res; stand-in waveform), Gaussian noise", scenarios={})
    th = torch.from_numpy(_pe_walkers(batch, 7)).to(dev)
    for name in ("pe22", "pehm", "penet"):
        cfg = W.config(name)
        ctx, thp, h0, n = _noisy_context(torch, pes, cfg, 2026, batch)
        far = thp.clone()
        far[0, 4] = 1e12                      # D_L -> h ~ 0: log L = -<d|d>/2
        ctx.set_data(h0)
        snr = math.sqrt(-2.0 * float(ctx.loglike(far)[0]))
        ctx.set_data(n)
        nn = -2.0 * float(ctx.loglike(far)[0])
        ctx.set_data(h0 + n)
        L_inj = float(ctx.loglike(thp)[0])
        o1 = torch.empty(1, dtype=torch.float64, device=dev)
        t_one = np.mean([_time_ms(torch, lambda i=i: ctx.loglike(th[i:i + 1], o1), reps)
                         for i in range(n_single)])
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        t1 = th[:1].clone()
        with torch.cuda.stream(s):
            ctx.loglike(t1, o1)
        torch.cuda.current_stream().wait_stream(s)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            ctx.loglike(t1, o1)
        t_graph = _time_ms(torch, g.replay, 20)
        ob = torch.empty(batch, dtype=torch.float64, device=dev)
        ctx.autotune(th)
        t_batch = _time_ms(torch, lambda: ctx.loglike(th, ob), reps)
        ctx.close()
        n_dof = 2 * 3 * len(cfg["detectors"]) * cfg["n_bins"]
        out["scenarios"][name] = dict(
            detectors=[d["kind"] for d in cfg["detectors"]], modes=len(cfg["modes"]), n_bins=cfg["n_bins"],
            snr=round(snr, 1), noise_nn_over_dof=round(nn / n_dof, 4),
            loglike_at_injection_over_minus_nn_half=round(L_inj / (-0.5 * nn), 12),
            one_sample_ms=round(float(t_one), 4), one_sample_graph_ms=round(t_graph, 4),
            batch=batch, batch_ms=round(t_batch, 3),
            evals_per_s_one_sample=round(1e3 / float(t_one), 1),
            evals_per_s_batched=round(batch / (t_batch * 1e-3), 1))
    sweep = []
    for p in range(12, 22):
        T = W.PE_DT * 2 ** p
        cfg = dict(detectors=[W.LISA], modes=W.MODES_HM, walkers=batch, name=f"series_2^{p}",
                   **W.grid_series(T))
        ctx, thp, h0, n = _noisy_context(torch, pes, cfg, 2027, batch)
        ctx.set_data(h0 + n)
        o1 = torch.empty(1, dtype=torch.float64, device=dev)
        t_one = np.mean([_time_ms(torch, lambda i=i: ctx.loglike(th[i:i + 1], o1), reps)
                         for i in range(n_single)])
        ob = torch.empty(batch, dtype=torch.float64, device=dev)
        t_batch = _time_ms(torch, lambda: ctx.loglike(th, ob), reps)
        ctx.set_precision(32)      # the paper's second precision (Fig. fig_cost)
        t_one32 = np.mean([_time_ms(torch, lambda i=i: ctx.loglike(th[i:i + 1], o1), reps)
                           for i in range(n_single)])
        t_batch32 = _time_ms(torch, lambda: ctx.loglike(th, ob), reps)
        ctx.close()
        sweep.append(dict(series_samples=2 ** p, duration_days=round(T / W.DAY_S, 2), n_bins=cfg["n_bins"],
                          one_sample_ms=round(float(t_one), 4),
                          batched_ms_per_sample=round(t_batch / batch, 5),
                          one_sample_ms_fp32=round(float(t_one32), 4),
                          batched_ms_per_sample_fp32=round(t_batch32 / batch, 5)))
    out["cost_vs_bins"] = sweep
    return out


def fp32_leg(torch, pes, steps, L64_ref=None):
    """The headline workload (LISA-like, five modes, 2^20 bins, 4096 prior
    walkers) with the single-precision kernels: evals/s at the autotuned
    tuning, and the deviation from the FP64 path on the same batch relative to
    max(|L|, <d|d>/2)."""
    cfg = W.config("cfg1")
    B = cfg["walkers"]
    dev = torch.device("cuda:0")
    ctx = pes.Context(cfg)
    ctx.reserve(B)
    th0 = torch.from_numpy(W.THETA0[None, :].copy()).to(dev)
    ctx.set_data(ctx.response(th0)[0].clone())
    theta = torch.from_numpy(W.draw_walkers(B, stream=1)).to(dev)
    out = torch.empty(B, dtype=torch.float64, device=dev)
    far = th0.clone()
    far[0, 4] = 1e12
    sigma = -float(ctx.loglike(far)[0])           # <d|d>/2
    ctx.autotune(theta)
    t64 = _time_ms(torch, lambda: ctx.loglike(theta, out), steps)
    L64 = out.cpu().numpy().copy()
    ctx.set_precision(32)
    _, tuning = ctx.autotune(theta)
    ctx.timing(True)
    t32 = _time_ms(torch, lambda: ctx.loglike(theta, out), steps)
    kern_ms, launches = ctx.timing_read()
    ctx.timing(False)
    L32 = out.cpu().numpy()
    ctx.close()
    rel = np.abs(L32 - L64) / np.maximum(np.abs(L64), sigma)
    return dict(workload="LISA-like, 5 modes, 2^20 bins (df=1/yr), 4096 walkers, noise-free injection",
                tuning=tuning, ms_per_call=round(t32, 3), evals_per_s=round(B / (t32 * 1e-3), 1),
                kernel_ms=round(kern_ms / launches, 3),
                fp64_ms_per_call_same_run=round(t64, 3), speedup_over_fp64=round(t64 / t32, 3),
                max_rel_dev_from_fp64=float(f"{rel.max():.3e}"),
                median_rel_dev_from_fp64=float(f"{np.median(rel):.3e}"))


def kepler_leg(torch, pes, steps):
    """The headline workload with the heliocentric detector on exact Kepler
    ellipses (arms flexing at order e^2 AU) instead of the first-order
    triangle: evals/s at the autotuned tuning and the cost relative to the
    first-order orbit in the same run, in FP64 and with the single-precision
    kernels (and their deviation from FP64 relative to max(|L|, <d|d>/2)),
    each also at the context's default tuning (the autotuner's gain);
    then the derivatives on both orbits (Fisher matrices at 256 points,
    forward- and reverse-mode gradients at 1024 walkers)."""
    out = {}
    for orbit in ("first_order", "kepler"):
        cfg = W.config("cfg1")
        cfg["detectors"] = [dict(d, orbit=orbit) for d in cfg["detectors"]]
        B = cfg["walkers"]
        dev = torch.device("cuda:0")
        ctx = pes.Context(cfg)
        ctx.reserve(B)
        th0 = torch.from_numpy(W.THETA0[None, :].copy()).to(dev)
        ctx.set_data(ctx.response(th0)[0].clone())
        theta = torch.from_numpy(W.draw_walkers(B, stream=1)).to(dev)
        o = torch.empty(B, dtype=torch.float64, device=dev)
        far = th0.clone()
        far[0, 4] = 1e12
        sigma = -float(ctx.loglike(far)[0])           # <d|d>/2
        default_ms = _time_ms(torch, lambda: ctx.loglike(theta, o), steps)   # the context's default tuning
        _, tuning = ctx.autotune(theta)
        out[orbit] = dict(ms_per_call=round(_time_ms(torch, lambda: ctx.loglike(theta, o), steps), 3),
                          tuning=tuning, default_tuning_ms=round(default_ms, 3))
        L64 = o.cpu().numpy().copy()
        ctx.set_precision(32)
        ctx.set_tuning(1, 16, 0)
        default32_ms = _time_ms(torch, lambda: ctx.loglike(theta, o), steps)
        _, tuning32 = ctx.autotune(theta)
        out[orbit]["fp32_ms_per_call"] = round(_time_ms(torch, lambda: ctx.loglike(theta, o), steps), 3)
        out[orbit]["fp32_tuning"] = tuning32
        out[orbit]["fp32_default_tuning_ms"] = round(default32_ms, 3)
        rel = np.abs(o.cpu().numpy() - L64) / np.maximum(np.abs(L64), sigma)
        out[orbit]["fp32_max_rel_dev_from_fp64"] = float(f"{rel.max():.3e}")
        ctx.set_precision(64)
        thf = theta[:256].contiguous()
        thg = theta[:1024].contiguous()
        ctx.set_grad_method("forward")
        out[orbit]["fisher_ms"] = round(_time_ms(torch, lambda: ctx.fisher(thf), 2), 3)
        out[orbit]["grad_forward_ms"] = round(_time_ms(torch, lambda: ctx.grad(thg), 1), 3)
        ctx.set_grad_method("adjoint")
        out[orbit]["grad_adjoint_ms"] = round(_time_ms(torch, lambda: ctx.grad(thg), 3), 3)
        ctx.close()
    k, f = out["kepler"], out["first_order"]
    return dict(workload="LISA-like on exact Kepler ellipses, 5 modes, 2^20 bins (df=1/yr), 4096 walkers, "
                         "noise-free injection; Fisher at 256 and gradients at 1024 of them",
                ms_per_call=k["ms_per_call"], evals_per_s=round(4096 / (k["ms_per_call"] * 1e-3), 1),
                tuning=k["tuning"], first_order_ms_per_call_same_run=f["ms_per_call"],
                cost_over_first_order=round(k["ms_per_call"] / f["ms_per_call"], 3),
                default_tuning_ms=k["default_tuning_ms"],
                autotune_gain=round(k["default_tuning_ms"] / k["ms_per_call"], 3),
                fp32_default_tuning_ms=k["fp32_default_tuning_ms"],
                fp32_autotune_gain=round(k["fp32_default_tuning_ms"] / k["fp32_ms_per_call"], 3),
                fp32_ms_per_call=k["fp32_ms_per_call"], fp32_evals_per_s=round(4096 / (k["fp32_ms_per_call"] * 1e-3), 1),
                fp32_tuning=k["fp32_tuning"], fp32_first_order_ms_per_call=f["fp32_ms_per_call"],
                fp32_speedup_over_fp64=round(k["ms_per_call"] / k["fp32_ms_per_call"], 3),
                fp32_max_rel_dev_from_fp64=k["fp32_max_rel_dev_from_fp64"],
                fisher_ms=k["fisher_ms"], fisher_first_order_ms=f["fisher_ms"],
                grad_forward_ms=k["grad_forward_ms"], grad_forward_first_order_ms=f["grad_forward_ms"],
                grad_adjoint_ms=k["grad_adjoint_ms"], grad_adjoint_first_order_ms=f["grad_adjoint_ms"])


EXTRINSIC = (7, 8, 9, 10)   # lambda, beta, psi, t_c


def fisher_sampling_leg(torch, pes, B, n_steps, seed=21):
    """The extrinsic parameters (lambda, beta, psi, t_c) of the noise-free
    injection on the LISA-like 5-mode 2^20-bin likelihood, the intrinsic ones
    held at their injected values: the inverse of the Fisher matrix's
    extrinsic block (pes_fisher) against the covariance of a DE-MC run
    (pes_loglike) started from that Gaussian, second half of the chain."""
    cfg = W.config("cfg1")
    dev = torch.device("cuda:0")
    ctx = pes.Context(cfg)
    th0 = torch.from_numpy(W.THETA0[None, :].copy()).to(dev)
    ctx.set_data(ctx.response(th0)[0].clone())
    S = list(EXTRINSIC)
    F = ctx.fisher(th0).cpu().numpy()[0]
    C_f = np.linalg.inv(F[np.ix_(S, S)])
    C_f = 0.5 * (C_f + C_f.T)
    prior = _prior_spec()
    for j in range(11):
        if j not in S:
            prior[j] = ("fixed", W.THETA0[j], W.THETA0[j])
    rng = np.random.default_rng(seed)
    start = np.tile(W.THETA0, (B, 1))
    start[:, S] = rng.multivariate_normal(W.THETA0[S], C_f, size=B)
    smp = pes.Sampler(ctx, prior, B, seed, chain_len=n_steps)
    smp.set_state(torch.from_numpy(start).to(dev))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    smp.step(n_steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    acc = smp.state()[2].cpu().numpy().sum() / (B * n_steps)
    ch = smp.read_chain().cpu().numpy()[n_steps // 2:]
    smp.close()
    ctx.close()
    from paper_2602_12011_amd import diagnostics as D
    x = ch[:, :, S].reshape(-1, len(S))
    C_s = np.cov(x.T)
    sd_f, sd_s = np.sqrt(np.diag(C_f)), np.sqrt(np.diag(C_s))
    r_f = C_f / np.outer(sd_f, sd_f)
    r_s = C_s / np.outer(sd_s, sd_s)
    iu = np.triu_indices(len(S), 1)
    snr = float(np.sqrt(max(F[4, 4], 0.0)) * W.THETA0[4])   # d ln h / d ln D_L = -1: sqrt(F_DD) D_L
    return dict(workload="LISA-like, 5 modes, 2^20 bins, noise-free injection; lambda, beta, psi, t_c free, "
                         f"the rest fixed; {B} walkers, {n_steps} DE steps",
                snr=round(snr, 1), seconds=round(dt, 2), acceptance=round(float(acc), 4),
                rhat_max=round(float(D.gelman_rubin(ch[:, :, S]).max()), 4),
                parameters=["lambda", "beta", "psi", "t_c"],
                sd_fisher=[float(f"{v:.4g}") for v in sd_f], sd_sampled=[float(f"{v:.4g}") for v in sd_s],
                sd_ratio_sampled_over_fisher=[round(float(v), 4) for v in sd_s / sd_f],
                corr_fisher=[round(float(v), 4) for v in r_f[iu]],
                corr_sampled=[round(float(v), 4) for v in r_s[iu]],
                mean_offset_in_fisher_sd=[round(float(v), 3) for v in (x.mean(axis=0) - W.THETA0[S]) / sd_f])


def _prior_spec():
    spec = []
    for name in W.PARAM_NAMES:
        kind, lo, hi = W.PRIOR[name]
        if name in ("phi_c", "lambda", "psi"):
            kind = "periodic"
        spec.append((kind, lo, hi))
    return spec


def _fisher_start(ctx, torch, B, seed):
    """Walkers from the Fisher Gaussian at the injection (regularized by the
    prior widths), clipped to the prior box."""
    dev = torch.device("cuda:0")
    th0 = torch.from_numpy(W.THETA0[None, :].copy()).to(dev)
    F = ctx.fisher(th0).cpu().numpy()[0]
    w = W.prior_widths()
    C = np.linalg.inv(F + np.diag(1.0 / w ** 2))
    C = 0.5 * (C + C.T)
    rng = np.random.default_rng(seed)
    x = rng.multivariate_normal(W.THETA0, C, size=B)
    lo = np.array([W.PRIOR[n][1] for n in W.PARAM_NAMES])
    hi = np.array([W.PRIOR[n][2] for n in W.PARAM_NAMES])
    eps = 1e-9 * (hi - lo)
    return np.clip(x, lo + eps, hi - eps)


def flow_leg(torch, pes, fit_steps=200, batch=4096, rows=1 << 17, n_eval=16384):
    """The learned proposal's network on its own: Adam steps of the NLL fit at
    the ESS leg's minibatch (4096 rows), and one normalizing (log q) and one
    sampling pass over 16384 rows (the ensemble of the config-4 sampler), on
    synthetic 11-D training rows (a correlated Gaussian bent along two
    coordinates).  All products run on the BF16 matrix-core GEMM."""
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(5)
    A = rng.normal(size=(11, 11)) / 4 + np.eye(11)
    x = rng.normal(size=(rows, 11)) @ A.T
    x[:, 1] += 0.5 * x[:, 0] ** 2
    x[:, 3] -= 0.3 * x[:, 2] ** 2
    tr = torch.from_numpy(x).to(dev)
    flow = pes.Flow(seed=11)
    flow.fit(tr, steps=5, batch=batch, lr=1e-3, seed=1)          # warm-up (workspace, first launches)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss = flow.fit(tr, steps=fit_steps, batch=batch, lr=1e-3, seed=2)
    torch.cuda.synchronize()
    t_fit = time.perf_counter() - t0
    ev = tr[:n_eval].contiguous()
    t_fwd = _time_ms(torch, lambda: flow.forward(ev), 20)
    z = torch.randn((n_eval, 11), dtype=torch.float64, device=dev, generator=torch.Generator(device=dev).manual_seed(3))
    t_inv = _time_ms(torch, lambda: flow.inverse(z), 20)
    flow.close()
    first_last = [float(loss[0]), float(loss[-1])] if hasattr(loss, "__len__") else None
    return dict(workload=f"8 coupling layers, width 256; fit minibatch {batch} rows of {rows} synthetic 11-D rows; "
                         f"passes over {n_eval} rows",
                fit_steps=fit_steps, ms_per_fit_step=round(t_fit / fit_steps * 1e3, 3),
                forward_ms=round(t_fwd, 3), inverse_ms=round(t_inv, 3), fit_loss_first_last=first_last)


def ess_leg(torch, pes, B, n_pilot, n_collect, n_run, fit_steps, tau=1.1, fit_batch=4096, ref_walkers=1024,
            n_ref=3000):
    """ESS/s of the plain DE-MC sampler against the mixture with the learned
    flow (p_flow 0.9, temperature tau) on the three-detector network with five
    modes at 2^20 bins (cfg4), B walkers.

    A plain DE pilot from the Fisher start burns in for n_pilot steps; the
    states of its last n_collect steps (every walker, repeats included, 10% of
    the walkers held out) train the flow.  Both arms then run n_run steps from
    the pilot's end state.  The reference is a long plain run of ref_walkers
    walkers from the same state (n_ref steps, second half, every 10th step).
    Accuracy of an arm: the largest per-parameter two-sample KS distance of
    its second-half draws from the reference; the bound is 1.5 times the KS
    distance between the reference's two walker halves (independent chains).
    Each arm's seconds to reach the bound are measured on a grid of run
    lengths (draws from the second half of the first t steps)."""
    from paper_2602_12011_amd import diagnostics as D
    cfg = W.config("cfg4")
    dev = torch.device("cuda:0")
    ctx = pes.Context(cfg)
    th0 = torch.from_numpy(W.THETA0[None, :].copy()).to(dev)
    ctx.set_data(ctx.response(th0)[0].clone())
    ctx.reserve(B)
    prior = _prior_spec()
    pilot = pes.Sampler(ctx, prior, B, 101, chain_len=n_collect)
    pilot.set_state(torch.from_numpy(_fisher_start(ctx, torch, B, 12)).to(dev))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(0, n_pilot, 50):
        pilot.step(min(50, n_pilot - k))
        torch.cuda.synchronize()
        print(f"[ess] pilot {min(k + 50, n_pilot)}/{n_pilot} steps, {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
    t_pilot = time.perf_counter() - t0
    ch = pilot.read_chain().cpu().numpy()                  # [n_collect, B, 11]
    state = pilot.state()[0].clone()
    pilot_acc = float(pilot.state()[2].cpu().numpy().sum()) / (B * n_pilot)
    pilot.close()
    rhat = float(D.gelman_rubin(ch).max())
    n_val_w = B // 10
    train = np.ascontiguousarray(ch[:, n_val_w:].reshape(-1, 11))
    val = np.ascontiguousarray(ch[:, :n_val_w].reshape(-1, 11))
    del ch
    # long plain reference
    ref = pes.Sampler(ctx, prior, ref_walkers, 404, chain_len=n_ref)
    ref.set_state(state[:ref_walkers].contiguous())
    t0 = time.perf_counter()
    for k in range(0, n_ref, 500):
        ref.step(min(500, n_ref - k))
        torch.cuda.synchronize()
        print(f"[ess] reference {min(k + 500, n_ref)}/{n_ref} steps, {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
    t_ref = time.perf_counter() - t0
    rch = ref.read_chain().cpu().numpy()[n_ref // 2::10]   # [n, ref_walkers, 11]
    ref.close()
    ref_draws = rch.reshape(-1, 11)
    h = ref_walkers // 2
    ks_split = max(D.ks_distance(rch[:, :h, j].ravel(), rch[:, h:, j].ravel()) for j in range(11))
    bound = 1.5 * ks_split
    # the learned proposal
    flow = pes.Flow(seed=7)
    tr = torch.from_numpy(train).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss = flow.fit(tr, steps=fit_steps, batch=fit_batch, lr=1e-3, seed=3)
    torch.cuda.synchronize()
    t_fit = time.perf_counter() - t0
    del tr
    nll_val = float(flow.nll_grad(torch.from_numpy(val[::8].copy()).to(dev))[0].cpu())
    flow.set_temperature(tau)
    results, chains = {}, {}
    for name, seed, use_flow in (("plain", 202, False), ("learned", 202, True)):
        smp = pes.Sampler(ctx, prior, B, seed, chain_len=n_run)
        smp.set_state(state)
        if use_flow:
            smp.set_flow(flow, 0.9)
        torch.cuda.synchronize()
        dt = 0.0
        for k in range(0, n_run, 50):   # chunks of 50 steps, so long runs report progress
            t0 = time.perf_counter()
            smp.step(min(50, n_run - k))
            torch.cuda.synchronize()
            dt += time.perf_counter() - t0
            print(f"[ess] {name}: {min(k + 50, n_run)}/{n_run} steps, {dt:.1f} s", file=sys.stderr, flush=True)
        acc = smp.state()[2].cpu().numpy().sum() / (B * n_run)
        chains[name] = smp.read_chain().cpu().numpy()
        smp.close()
        e = D.ess(chains[name])
        c = chains[name]
        draws = c[n_run // 2:].reshape(-1, 11)
        ks_j = [D.ks_distance(draws[:, j], ref_draws[:, j]) for j in range(11)]
        # seconds to reach the accuracy bound: second half of the first t steps
        t_acc = None
        for t in range(10, n_run + 1, 10):
            sub = c[t // 2:t, ::4].reshape(-1, 11)
            if max(D.ks_distance(sub[:, j], ref_draws[:, j]) for j in range(11)) <= bound:
                t_acc = t
                break
        results[name] = dict(seconds=round(dt, 3), acceptance=round(float(acc), 4),
                             ess_min=round(float(e.min()), 1), ess_per_s=round(float(e.min()) / dt, 2),
                             ks_vs_reference=round(max(ks_j), 4),
                             ks_per_parameter_vs_reference=[round(x, 4) for x in ks_j],
                             accuracy_ok=bool(max(ks_j) <= bound),
                             steps_to_accuracy=t_acc,
                             seconds_to_accuracy=None if t_acc is None else round(dt * t_acc / n_run, 3),
                             sd_ratio_vs_reference=[round(float(x), 3) for x in
                                                    draws.std(axis=0) / ref_draws.std(axis=0)])
    flow.close()
    ctx.close()
    gain = results["learned"]["ess_per_s"] / max(results["plain"]["ess_per_s"], 1e-30)
    both = results["learned"]["accuracy_ok"] and results["plain"]["accuracy_ok"]
    ta, tp = results["learned"]["seconds_to_accuracy"], results["plain"]["seconds_to_accuracy"]
    amort = results["learned"]["ess_min"] / (results["learned"]["seconds"] + t_fit)
    return dict(workload=f"LISA+Taiji+TianQin, 5 modes, 2^20 bins, {B} walkers, noise-free injection; "
                         f"{n_pilot}-step plain DE pilot, the states of its last {n_collect} steps train the "
                         f"flow; then {n_run} steps of each arm from the pilot's end",
                pilot_seconds=round(t_pilot, 2), pilot_acceptance=round(pilot_acc, 4),
                pilot_rhat_max=round(rhat, 4), train_rows=int(len(train)), heldout_rows=int(len(val)),
                fit_steps=fit_steps, fit_batch=fit_batch, fit_seconds=round(t_fit, 2),
                fit_loss_first_last=[round(float(loss[0]), 3), round(float(loss[-1]), 3)],
                heldout_nll=round(nll_val, 3), temperature=tau,
                plain=results["plain"], learned=results["learned"],
                gain=round(gain, 2), gain_at_matched_accuracy=round(gain, 2) if both else None,
                seconds_to_accuracy_ratio=(round(tp / ta, 2) if (ta and tp) else None),
                learned_ess_per_s_with_training=round(amort, 2),
                reference=dict(walkers=ref_walkers, steps=n_ref, seconds=round(t_ref, 2),
                               draws=int(len(ref_draws)), ks_between_walker_halves=round(ks_split, 4)),
                accuracy_bound=round(bound, 4))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-sample", type=int, default=48)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tuning", default=None,
                    help="bins_per_lane,walkers_per_group,blocks_per_cu (skips the autotuner)")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline measurement (no extra legs)")
    ap.add_argument("--extras", default="derivatives,graph,config2,fp32,kepler,fisher_sampling,paper_pe,flow,ess",
                    help="comma list of the extra legs to run after the headline")
    ap.add_argument("--ess-walkers", type=int, default=16384)
    ap.add_argument("--ess-pilot", type=int, default=300)
    ap.add_argument("--ess-collect", type=int, default=72,
                    help="last pilot steps whose states (all walkers) train the flow")
    ap.add_argument("--ess-steps", type=int, default=150)
    ap.add_argument("--ess-fit-steps", type=int, default=1000)
    ap.add_argument("--ess-ref-walkers", type=int, default=1024)
    ap.add_argument("--ess-ref-steps", type=int, default=3000)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device copy (for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps(dict(copy_bytes=src.numel() * 8, launches=3)))
        return 0
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(walkers are independent: N GPUs would each run their own batch).", file=sys.stderr)
        return 2

    import torch
    from paper_2602_12011_amd import pes

    cfg = W.config("cfg1")
    B = cfg["walkers"]
    theta_np = W.draw_walkers(B, stream=1)
    dev = torch.device("cuda:0")
    ctx = pes.Context(cfg)
    ctx.reserve(B)
    th0 = torch.from_numpy(W.THETA0[None, :].copy()).to(dev)
    data = ctx.response(th0)[0].clone()
    ctx.set_data(data)
    theta = torch.from_numpy(theta_np).to(dev)
    out = torch.empty(B, dtype=torch.float64, device=dev)
    tuning = ctx.get_tuning()
    if args.tuning:
        ctx.set_tuning(*[int(x) for x in args.tuning.split(",")])
        tuning = ctx.get_tuning()
    elif not args.no_autotune:
        _, tuning = ctx.autotune(theta)      # untimed: picks the kernel tuning for this shape
    for _ in range(args.warmup):
        ctx.loglike(theta, out)
    torch.cuda.synchronize()
    ctx.timing(True)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(args.steps):
        ctx.loglike(theta, out)
    stop.record()
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    kern_ms, launches = ctx.timing_read()
    ctx.timing(False)
    L = out.cpu().numpy()
    assert np.all(np.isfinite(L)), "non-finite log-likelihoods"
    ms_per_step = total_ms / args.steps
    value = B / (ms_per_step * 1e-3)

    flops, n_mode, n_wbd = algorithmic_flops(cfg, theta_np)
    kern_s = kern_ms / launches * 1e-3
    achieved = flops / kern_s / 1e12
    roofline = dict(bound="alu", achieved=round(achieved, 3), peak=PEAK_FP64_VECTOR_TFLOPS,
                    unit="TFLOP/s", frac=round(achieved / PEAK_FP64_VECTOR_TFLOPS, 4),
                    traffic=measured_traffic(tuning),
                    kernel="loglike_kernel", kernel_ms=round(kern_ms / launches, 4),
                    flops_per_launch=flops)

    rec = dict(metric=METRIC, value=round(value, 1), unit="logL evals/s", n_gpus=1,
               steps=args.steps, warmup=args.warmup, ms_per_step=round(ms_per_step, 4),
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f64",
               data="synthetic",
               config=dict(workload="LISA-like, 5 modes, 2^20 bins (df=1/yr), 4096 walkers, "
                                    "noise-free injection",
                           walkers=B, n_bins=cfg["n_bins"], modes=len(cfg["modes"]),
                           detectors=[d["kind"] for d in cfg["detectors"]],
                           mode_units=n_mode, wbd_units=n_wbd, tuning=tuning),
               roofline=roofline)
    ctx.close()
    if not args.no_cpu:
        threads = min(16, os.cpu_count() or 1)
        rec["cpu_baseline"] = cpu_baseline(cfg, theta_np, args.cpu_sample, threads)
    extras = [] if args.no_extras else [x for x in args.extras.split(",") if x]
    if "derivatives" in extras:
        print("[bench] derivatives", file=sys.stderr, flush=True)
        rec["derivatives"] = derivative_leg(torch, pes, 3)
    if "graph" in extras:
        print("[bench] sampler graph", file=sys.stderr, flush=True)
        rec["sampler_graph"] = graph_leg(torch, pes, 50)
    if "config2" in extras:
        print("[bench] config 2 schedules", file=sys.stderr, flush=True)
        rec["config2"] = config2_leg(torch, pes, 3)
    if "fp32" in extras:
        print("[bench] single precision", file=sys.stderr, flush=True)
        rec["fp32"] = fp32_leg(torch, pes, 10)
    if "kepler" in extras:
        print("[bench] exact Kepler orbits", file=sys.stderr, flush=True)
        rec["kepler"] = kepler_leg(torch, pes, 10)
    if "fisher_sampling" in extras:
        print("[bench] Fisher vs sampling, extrinsic parameters", file=sys.stderr, flush=True)
        rec["fisher_sampling"] = fisher_sampling_leg(torch, pes, 1024, 1000)
    if "paper_pe" in extras:
        print("[bench] paper's PE workload", file=sys.stderr, flush=True)
        rec["paper_pe"] = paper_pe_leg(torch, pes)
    if "flow" in extras:
        print("[bench] learned proposal network", file=sys.stderr, flush=True)
        rec["flow"] = flow_leg(torch, pes)
    if "ess" in extras:
        print("[bench] ESS", file=sys.stderr, flush=True)
        rec["ess"] = ess_leg(torch, pes, args.ess_walkers, args.ess_pilot, args.ess_collect, args.ess_steps,
                             args.ess_fit_steps, ref_walkers=args.ess_ref_walkers, n_ref=args.ess_ref_steps)
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
