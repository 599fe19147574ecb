"""Pins of the flow reference (oracle/flow.py) against facts that do not come
from its own formulas: torch's BF16 conversion, the normal density of an
affine map, finite differences, the inverse, and Adam's first step."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import flow as F


def test_bf16_matches_torch_conversion():
    import torch
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(size=4000) * 10.0 ** rng.integers(-30, 30, size=4000),
                        [0.0, -0.0, 1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -7 + 2.0 ** -8,
                         -1.0 - 2.0 ** -8, 3.0e38, 1e-40]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(F.bf16(x), ref)
    # ties go to even
    assert F.bf16(np.float32(1.0 + 2.0 ** -8)) == 1.0
    assert F.bf16(np.float32(1.0 + 3 * 2.0 ** -8)) == 1.0 + 2.0 ** -6


def test_layout():
    assert F.n_params() == 562264
    for l in range(F.N_LAYERS):
        C, T = F.cond_set(l), F.trans_set(l)
        assert sorted(C + T) == list(range(F.D))
        assert len(C) == (6 if l % 2 == 0 else 5)
        if l % 2:
            assert T == F.cond_set(l - 1)
    # every coordinate is transformed by some layer, conditioned on by some other
    for i in range(F.D):
        assert any(i in F.trans_set(l) for l in range(F.N_LAYERS))


def test_identity_when_output_layer_is_zero():
    flat = F.init_params(3, scale_out=0.0)
    u = np.random.default_rng(2).normal(size=(50, 11))
    z, ld = F.forward(flat, u)
    assert np.array_equal(z, u) and np.all(ld == 0.0)
    lp = F.log_prob_u(flat, u)
    assert np.allclose(lp, stats.norm.logpdf(u).sum(axis=1), rtol=1e-14, atol=1e-13)


def test_constant_couplings_give_the_gaussian_of_an_affine_map():
    """W3 = 0: every layer shifts and scales its transformed coordinates by
    constants, so u is Gaussian with per-coordinate mean and scale that follow
    from composing the affine maps; the density must be scipy's normal pdf."""
    rng = np.random.default_rng(4)
    flat = F.init_params(5, scale_out=0.0).astype(np.float64)
    layers = F.unflatten(flat)
    a = np.ones(11)   # z = a u + c
    c = np.zeros(11)
    for l, p in enumerate(layers):
        T = F.trans_set(l)
        nt = len(T)
        sh = rng.uniform(-2, 2, size=nt)
        t = rng.uniform(-1, 1, size=nt)
        p["b3"][:nt] = sh
        p["b3"][nt:] = t
        s = 3.0 * np.tanh(sh / 3.0)
        a[T] = a[T] * np.exp(s)
        c[T] = c[T] * np.exp(s) + t
    u = rng.normal(size=(200, 11))
    lp = F.log_prob_u(flat, u)
    ref = stats.norm.logpdf(u, loc=-c / a, scale=1.0 / a).sum(axis=1)
    assert np.allclose(lp, ref, rtol=1e-12, atol=1e-11)


@pytest.mark.parametrize("rnd", [False, True])
def test_inverse_undoes_forward(rnd):
    flat = F.init_params(6, scale_out=0.3)
    u = np.random.default_rng(7).normal(size=(100, 11))
    z, ld = F.forward(flat, u, rnd)
    u2, ld2 = F.inverse(flat, z, rnd)
    assert np.allclose(u2, u, rtol=0, atol=1e-12)
    assert np.allclose(ld2, ld, rtol=0, atol=1e-12)
    assert np.abs(z - u).max() > 0.1   # a non-trivial map


def test_logdet_matches_finite_difference_jacobian():
    flat = F.init_params(8, scale_out=0.3)
    u0 = np.random.default_rng(9).normal(size=(3, 11))
    _, ld = F.forward(flat, u0, rnd=False)
    h = 1e-6
    for b in range(3):
        J = np.zeros((11, 11))
        for j in range(11):
            e = np.zeros((1, 11))
            e[0, j] = h
            zp, _ = F.forward(flat, u0[b:b + 1] + e, rnd=False)
            zm, _ = F.forward(flat, u0[b:b + 1] - e, rnd=False)
            J[:, j] = (zp - zm)[0] / (2 * h)
        sign, logabs = np.linalg.slogdet(J)
        assert sign > 0
        assert abs(logabs - ld[b]) < 1e-7


def test_nll_gradient_matches_finite_differences():
    flat = F.init_params(10, scale_out=0.3).astype(np.float64)
    rng = np.random.default_rng(11)
    u = rng.normal(size=(16, 11)) * 1.3 + 0.2
    nll, g = F.nll_and_grad(flat, u, rnd=False)
    # coordinates from every tensor of every layer
    idx, o = [], 0
    for l in range(F.N_LAYERS):
        for name, sh in F.shapes(l):
            k = int(np.prod(sh))
            idx.extend(int(i) for i in o + rng.choice(k, size=2, replace=False))
            o += k
    for i in idx:
        h = 1e-6 * max(1.0, abs(flat[i]))
        fp = flat.copy()
        fp[i] += h
        fm = flat.copy()
        fm[i] -= h
        d = (F.nll_and_grad(fp, u, rnd=False)[0] - F.nll_and_grad(fm, u, rnd=False)[0]) / (2 * h)
        assert abs(d - g[i]) <= 1e-6 * max(1.0, abs(d)), (i, d, g[i])


def test_nll_is_the_mean_negative_log_density():
    flat = F.init_params(12, scale_out=0.3)
    u = np.random.default_rng(13).normal(size=(40, 11))
    nll, _ = F.nll_and_grad(flat, u)
    assert math.isclose(nll, -F.log_prob_u(flat, u).mean(), rel_tol=1e-13)


def test_adam_first_step_and_convergence():
    rng = np.random.default_rng(14)
    g = rng.normal(size=100)
    p = np.zeros(100)
    m, v = np.zeros(100), np.zeros(100)
    F.adam_step(p, g, m, v, 1, lr=1e-3)
    # with bias correction the first step is lr g / (|g| + eps)
    assert np.allclose(p, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    # minimizes a convex quadratic
    target = rng.normal(size=100)
    p = np.zeros(100)
    m, v = np.zeros(100), np.zeros(100)
    for t in range(1, 3001):
        F.adam_step(p, 2.0 * (p - target), m, v, t, lr=1e-2)
    assert np.abs(p - target).max() < 1e-3


def test_whitened_identity_flow_is_the_multivariate_normal():
    """With the identity flow, q(theta) is the Gaussian N(mu, L L^T) of the
    whitening map (scipy's density)."""
    rng = np.random.default_rng(15)
    A = rng.normal(size=(11, 11))
    C = A @ A.T / 11 + 0.05 * np.eye(11)
    L = np.linalg.cholesky(C)
    mu = rng.normal(size=11) * 3
    flat = F.init_params(16, scale_out=0.0)
    th = rng.multivariate_normal(mu, C, size=300)
    lq = F.log_prob(flat, th, mu, L)
    ref = stats.multivariate_normal(mu, C).logpdf(th)
    assert np.allclose(lq, ref, rtol=1e-6, atol=1e-5)
    # standardize and unstandardize are inverse maps (up to the FP32 rounding of u)
    u = F.standardize(th, mu, L)
    assert np.allclose(F.unstandardize(u, mu, L), th, rtol=0, atol=1e-5 * np.abs(th).max())
    assert np.allclose(np.cov(u.T), np.linalg.inv(L) @ np.cov(th.T) @ np.linalg.inv(L).T, atol=1e-6)


def test_temperature_widens_the_gaussian():
    """Identity flow at temperature tau: q is N(mu, tau^2 L L^T)."""
    rng = np.random.default_rng(17)
    A = rng.normal(size=(11, 11))
    C = A @ A.T / 11 + 0.05 * np.eye(11)
    L = np.linalg.cholesky(C)
    mu = rng.normal(size=11)
    flat = F.init_params(18, scale_out=0.0)
    th = rng.multivariate_normal(mu, 2.0 * C, size=200)
    lq = F.log_prob(flat, th, mu, L, tau=1.4)
    ref = stats.multivariate_normal(mu, 1.96 * C).logpdf(th)
    assert np.allclose(lq, ref, rtol=1e-6, atol=1e-5)
