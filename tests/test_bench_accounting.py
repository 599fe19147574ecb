"""Host logic of bench.py's algorithmic FLOP count and utilisation figures."""
import numpy as np

import bench
from paper_2602_12011_amd import workloads as W


def test_paired_modes():
    # the second mode of each m rides on the first mode's unit
    assert bench.paired_modes([(2, 2), (2, 1), (3, 3), (3, 2), (4, 4)]) == {3}
    assert bench.paired_modes([(2, 2)]) == set()
    assert bench.paired_modes([(2, 2), (3, 2), (4, 2)]) == {1}


def test_bin_classes_follow_wavefronts():
    cfg = W.config("cfg1", n_bins=1000)
    cls = bench.bin_classes(cfg, W.LISA)
    # constant over each aligned 64-bin wavefront, non-decreasing in frequency
    assert np.all(np.ptp(cls[:960].reshape(-1, 64), axis=1) == 0)
    assert np.all(np.diff(cls) >= 0)
    # TianQin (L = 0.57 s): every bin of the 2^20 grid is short-range
    assert np.all(bench.bin_classes(W.config("cfg1"), W.TIANQIN) == 0)


def test_flops_counts_one_unit_per_pair():
    cfg = W.config("cfg1", n_bins=4096)
    th = W.draw_walkers(8, stream=3)
    f_all, n_mode, n_wb = bench.algorithmic_flops(cfg, th)
    ns, nmax = bench.mode_bin_counts(cfg, th)
    assert n_mode == ns.sum() and n_wb == nmax.sum()
    # removing the paired (3,2) mode removes exactly 19 flops per active bin of it
    cfg2 = dict(cfg, modes=[m for m in cfg["modes"] if m != (3, 2)])
    f_less, _, _ = bench.algorithmic_flops(cfg2, th)
    assert abs((f_all - f_less) - bench.FLOPS_PER_PAIRED_MODE * ns[:, 3].sum()) < 1e-6 * f_all


def test_schedule_utilisation_bounds():
    cfg = W.config("cfg2", n_bins=20000)
    th = W.draw_walkers(64, stream=4)
    uq = bench.schedule_utilisation(cfg, th, 512, False)
    ug = bench.schedule_utilisation(cfg, th, 512, True)
    assert 0 < ug[0] <= uq[0] <= 1 and 0 < ug[1] <= uq[1] <= 1
