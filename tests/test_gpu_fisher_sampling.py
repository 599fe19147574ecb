"""The Fisher matrix (forward-mode Jacobian + FP64 matrix cores) against
sampling (DE-MC on the exact log-likelihood): on the noise-free injection at
SNR ~1900 the posterior of the extrinsic parameters, the intrinsic ones held
fixed, is Gaussian to leading order with the inverse of the Fisher matrix's
extrinsic block as covariance (Sec. 2.2 and 3.3).  Two independently built
paths of the library have to agree: standard deviations within 5%,
correlations within 0.02, means within 0.1 standard deviations (the
sampling error of 512 walkers x 300 kept steps is below 1%)."""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

sys.path.insert(0, os.path.join(os.path.dirname(__file__), ".."))


def test_extrinsic_posterior_matches_inverse_fisher():
    import torch
    import bench
    from paper_2602_12011_amd import pes
    assert torch.cuda.is_available()
    print("[fisher-sampling] cfg1 grid, 512 walkers, 600 steps", flush=True)
    r = bench.fisher_sampling_leg(torch, pes, 512, 600)
    assert r["snr"] > 1000
    assert r["rhat_max"] < 1.01
    assert np.all(np.abs(np.array(r["sd_ratio_sampled_over_fisher"]) - 1.0) < 0.05), r
    assert np.all(np.abs(np.array(r["corr_sampled"]) - np.array(r["corr_fisher"])) < 0.02), r
    assert np.all(np.abs(r["mean_offset_in_fisher_sd"]) < 0.1), r
