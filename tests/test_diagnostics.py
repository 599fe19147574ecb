"""Chain diagnostics (host code) against processes with known answers."""
import numpy as np
from scipy import stats

from paper_2602_12011_amd import diagnostics as D


def _ar1(rho, T, B, d, seed):
    rng = np.random.default_rng(seed)
    x = np.zeros((T, B, d))
    x[0] = rng.normal(size=(B, d)) / np.sqrt(1 - rho * rho)
    for t in range(1, T):
        x[t] = rho * x[t - 1] + rng.normal(size=(B, d))
    return x


def test_integrated_time_of_ar1():
    # AR(1): tau = (1 + rho) / (1 - rho)
    for rho in (0.0, 0.5, 0.9):
        tau = D.integrated_time(_ar1(rho, 4000, 16, 2, seed=int(10 * rho)))
        exact = (1 + rho) / (1 - rho)
        assert np.all(np.abs(tau - exact) < 0.1 * exact), (rho, tau, exact)


def test_ess_scales_with_walkers_and_length():
    x = _ar1(0.8, 3000, 8, 1, seed=3)
    e = D.ess(x)[0]
    assert abs(e - 8 * 3000 / 9.0) < 0.15 * 8 * 3000 / 9.0


def test_gelman_rubin():
    x = _ar1(0.5, 1000, 64, 3, seed=4)
    assert np.all(D.gelman_rubin(x) < 1.01)
    x[:, :16, 0] += 2.0   # one group off: R^2 = 1 + 1 / var(x) = 1.75
    r = D.gelman_rubin(x)
    assert abs(r[0] - np.sqrt(1.75)) < 0.03 and np.all(r[1:] < 1.01)


def test_ks_distance_matches_scipy():
    rng = np.random.default_rng(5)
    a, b = rng.normal(size=700), rng.normal(0.1, 1.2, size=900)
    assert abs(D.ks_distance(a, b) - stats.ks_2samp(a, b).statistic) < 1e-12

