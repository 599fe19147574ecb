"""Pins of the sampler reference (CPU): Philox4x32-10 against its published
known-answer vectors, and the DE-MC chains against the exact marginals of a
correlated 11-D Gaussian target."""
import math
import os

import numpy as np
import pytest
from scipy import stats

from oracle import sampler as S

HERE = os.path.dirname(os.path.abspath(__file__))


def kat_vectors():
    out = []
    for line in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(x, 16) for x in line.split()]
        out.append((tuple(w[:4]), tuple(w[4:6]), tuple(w[6:10])))
    return out


@pytest.mark.parametrize("vec", kat_vectors())
def test_philox_known_answers(vec):
    ctr, key, expect = vec
    assert S.philox4x32_10(ctr, key) == expect


def test_uniforms_in_open_interval():
    assert 0.0 < S.u01(0, 0) < 1e-15
    assert S.u01(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53


def test_de_sampler_recovers_gaussian_marginals():
    rng = np.random.default_rng(4)
    d = 11
    A = rng.normal(size=(d, d))
    C = A @ A.T / d + 0.2 * np.eye(d)
    Ci = np.linalg.inv(C)
    mu = rng.normal(size=d)

    def loglike(th):
        r = np.atleast_2d(th) - mu
        return -0.5 * np.einsum("bi,ij,bj->b", r, Ci, r)

    prior = [("uniform", -50.0, 50.0)] * d
    B = 128
    theta0 = mu + rng.normal(size=(B, d)) * 3.0
    smp = S.DESampler(loglike, prior, theta0, seed=0x1234)
    for _ in range(400):
        smp.step()
    draws = []
    for n in range(400):
        smp.step()
        if n % 25 == 0:
            draws.append(smp.theta.copy())
    draws = np.concatenate(draws)
    assert 0.1 < smp.accepts.sum() / (B * 800) < 0.6
    for j in range(d):
        p = stats.kstest(draws[:, j], "norm", args=(mu[j], math.sqrt(C[j, j]))).pvalue
        assert p > 1e-3, (j, p)
