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


def _gaussian(seed, d=11):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(d, d))
    C = A @ A.T / d + 0.2 * np.eye(d)
    return rng, rng.normal(size=d), C


def test_flow_proposal_equal_to_the_target_is_always_accepted():
    """Independence MH with q = pi accepts every move: the identity flow with
    mu, sigma of an axis-aligned Gaussian target is that target."""
    from oracle import flow as F
    rng = np.random.default_rng(5)
    d = 11
    m = rng.normal(size=d)
    s = rng.uniform(0.5, 2.0, size=d)

    def loglike(th):
        r = (np.atleast_2d(th) - m) / s
        return -0.5 * (r * r).sum(axis=1)

    prior = [("uniform", -80.0, 80.0)] * d
    flat = F.init_params(1, scale_out=0.0)
    B = 32
    smp = S.DESampler(loglike, prior, m + s * rng.normal(size=(B, d)), seed=77, flow=(flat, m, s, 1.0))
    for _ in range(20):
        smp.step()
    assert smp.accepts.sum() == B * 20


def _flow_mixture_draws(flip=False):
    """Mixture chains (p_flow 0.9) on an axis-aligned Gaussian with a flow that
    is a near-identity map of a shifted, widened Gaussian; the walkers'
    states at snapshots 30 steps apart (the flow moves are independence
    proposals accepted about a third of the time, so the snapshots are
    nearly independent)."""
    from oracle import flow as F
    rng = np.random.default_rng(6)
    d = 11
    m = rng.normal(size=d)
    s = rng.uniform(0.5, 2.0, size=d)

    def loglike(th):
        r = (np.atleast_2d(th) - m) / s
        return -0.5 * (r * r).sum(axis=1)

    prior = [("uniform", -50.0, 50.0)] * d
    flat = F.init_params(2, scale_out=0.05)
    B = 256
    smp = S.DESampler(loglike, prior, m + rng.normal(size=(B, d)) * s, seed=0x4321,
                      flow=(flat, m + 0.2 * s, 1.3 * s, 0.9))
    if flip:   # a planted mistake: the Hastings term with the wrong sign
        orig = smp._flow_mix
        smp._flow_mix = lambda *a: (lambda pq: (pq[0], -pq[1]))(orig(*a))
    for _ in range(60):
        smp.step()
    draws = []
    for n in range(4):
        for _ in range(30):
            smp.step()
        draws.append(smp.theta.copy())
    return np.concatenate(draws), m, s, smp.accepts.sum() / (B * smp.step_no)


def _marginals_ok(draws, m, s):
    ps = [stats.kstest(draws[:, j], "norm", args=(m[j], s[j])).pvalue for j in range(len(m))]
    return min(ps) > 1e-3, ps


def test_flow_mixture_recovers_gaussian_marginals():
    draws, m, s, rate = _flow_mixture_draws()
    assert 0.2 < rate < 0.6
    ok, ps = _marginals_ok(draws, m, s)
    assert ok, ps
    assert np.all(np.abs(draws.mean(axis=0) - m) / s < 0.1)


def test_flow_mixture_check_detects_a_wrong_hastings_term():
    draws, m, s, _ = _flow_mixture_draws(flip=True)
    assert not _marginals_ok(draws, m, s)[0]
