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
# geocentric orbit, short or long sinc fit -- and per active (walker, bin,
# detector) for the TDI combination and the inner products.  The C^2 taper
# (the last 10% below each cutoff) is not counted.
FLOPS_PER_MODE_UNIT = {("helio", False): 459, ("geo", False): 485,
                       ("helio", True): 487, ("geo", True): 513}
FLOPS_PER_WBD_UNIT = 83
MF_ISCO = 6.0 ** -1.5 / math.pi
MSUN_S = 4.925490947641267e-6


def active_units(cfg, theta):
    """(mode units, walker-bin units) per detector that one pes_loglike evaluates."""
    N, f0, df = cfg["n_bins"], cfg["f0"], cfg["df"]
    M = theta[:, 0] * MSUN_S
    n_mode = np.zeros(len(theta))
    n_any = np.zeros(len(theta))
    for (l, m) in cfg["modes"]:
        fcut = 0.5 * m * MF_ISCO / M
        n = np.clip(np.ceil((fcut - f0) / df), 0, N)
        n_mode += n
        n_any = np.maximum(n_any, n)
    return float(n_mode.sum()), float(n_any.sum())


def algorithmic_flops(cfg, theta):
    n_mode, n_wb = active_units(cfg, theta)
    f_max = cfg["f0"] + (cfg["n_bins"] - 1) * cfg["df"]
    total = 0.0
    for d in cfg["detectors"]:
        L = d["arm_m"] / 299792458.0
        long_sinc = (2 * math.pi * f_max * L) ** 2 > 4.9
        orbit = "geo" if d["kind"] == "tianqin" else "helio"
        total += FLOPS_PER_MODE_UNIT[(orbit, long_sinc)] * n_mode + FLOPS_PER_WBD_UNIT * n_wb
    nd = len(cfg["detectors"])
    return total, n_mode * nd, n_wb * nd


KERNEL_SOURCES = ("pes_eval.hpp", "pes_kernels.hip", "pes_math.hpp", "pes_poly.hpp",
                  "pes_layout.hpp", "pes_launch.hpp")
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
    vals = {}
    for line in text.splitlines():
        if ":" in line and line.split(":")[0].strip() in (
                "traffic_bytes_per_launch", "kernel_sources_sha256_16", "tuning"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    tun = f"{tuning['bins_per_lane']},{tuning['walkers_per_group']},{tuning['blocks_per_cu']}"
    if vals.get("kernel_sources_sha256_16") != kernel_source_hash() or vals.get("tuning") != tun:
        return None
    return float(vals["traffic_bytes_per_launch"])


def cpu_baseline(cfg, theta, n_sample, threads):
    import oracle
    d = oracle.response(cfg, W.THETA0)
    sample = theta[:n_sample]
    oracle.loglike(cfg, d, sample[:1], nthreads=threads)   # load + warm
    t0 = time.perf_counter()
    oracle.loglike(cfg, d, sample, nthreads=threads)
    dt = time.perf_counter() - t0
    return dict(value=n_sample / dt, unit="logL evals/s", cores=threads, kind="oracle",
                sample=f"{n_sample} of the {len(theta)} walkers, full {cfg['n_bins']}-bin grid, "
                       f"5 modes, {dt:.1f} s wall")


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
    if not args.no_cpu:
        threads = min(16, os.cpu_count() or 1)
        rec["cpu_baseline"] = cpu_baseline(cfg, theta_np, args.cpu_sample, threads)
    print(json.dumps(rec), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
