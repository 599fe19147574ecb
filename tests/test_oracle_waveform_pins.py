"""Pins of the oracle's waveform stand-in (CPU only): eq. (eq_tf) against a
finite difference of the phase, the SPA mode scaling, the textbook
restricted-PN amplitude and the Newtonian chirp time."""
import math

import numpy as np
import pytest

from paper_2602_12011_amd import workloads as W

MSUN_S = 4.925490947641267e-6
GPC_S = 3.085677581491367e25 / 299792458.0


def _theta(**kw):
    th = W.THETA0.copy()
    for k, v in kw.items():
        th[W.PARAM_NAMES.index(k)] = v
    return th


@pytest.mark.parametrize("lm", W.MODES_HM)
@pytest.mark.parametrize("Mtot", [1e5, 1e6, 1e7])
def test_tf_is_phase_derivative(orc, lm, Mtot):
    """Eq. (eq_tf): t_f = (1/2 pi) dPsi/df (t_c = 0 so that t_f is the chirp time)."""
    l, m = lm
    th = _theta(M_tot=Mtot, q=0.4, chi1=0.6, chi2=-0.3, t_c=0.0)
    M = Mtot * MSUN_S
    fcut = (m / 2) * 6 ** -1.5 / math.pi / M
    f = np.geomspace(1e-4 * fcut / 3.3e-2, 0.85 * fcut, 7)
    _, _, tf = orc.mode(th, l, m, f)
    h = 1e-6 * f
    _, pp, _ = orc.mode(th, l, m, f + h)
    _, pm, _ = orc.mode(th, l, m, f - h)
    tf_fd = (pp - pm) / (2 * h) / (2 * math.pi)
    np.testing.assert_allclose(tf, tf_fd, rtol=1e-7)


@pytest.mark.parametrize("lm", W.MODES_HM[1:])
def test_spa_mode_scaling(orc, lm):
    """t_f^{lm}(f) = t_f^{22}(2f/m) and Psi_lm(f) = (m/2) Psi_22(2f/m) up to the
    f-linear t_c term and the constants -(m/2) phi_c - pi/4."""
    l, m = lm
    th = _theta(q=0.3, chi1=0.5, chi2=0.2)
    f = np.geomspace(2e-4, 3e-3, 11) * m / 2
    _, psi_lm, tf_lm = orc.mode(th, l, m, f)
    _, psi_22, tf_22 = orc.mode(th, 2, 2, 2 * f / m)
    np.testing.assert_allclose(tf_lm, tf_22, rtol=1e-14)
    tc, phic = th[10], th[6]
    lhs = psi_lm - 2 * math.pi * f * tc + (m / 2) * phic + math.pi / 4
    rhs = (m / 2) * (psi_22 - 2 * math.pi * (2 * f / m) * tc + phic + math.pi / 4)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-9)


def test_restricted_pn_amplitude_22(orc):
    """|h_+| = sqrt(5/24) pi^{-2/3} Mc^{5/6} f^{-7/6} (1 + cos^2 i) / (2 D_L)."""
    th = _theta(q=0.7, iota=0.9, D_L=3.0)
    f = np.geomspace(1e-4, 3e-3, 9)
    h, _, _ = orc.mode(th, 2, 2, f)
    Kp, _ = orc.pol_coeffs(2, 2, th[5])
    M = th[0] * MSUN_S
    eta = th[1] / (1 + th[1]) ** 2
    Mc = eta ** 0.6 * M
    ref = (math.sqrt(5 / 24) * math.pi ** (-2 / 3) * Mc ** (5 / 6) * f ** (-7 / 6)
           * (1 + math.cos(th[5]) ** 2) / (2 * th[4] * GPC_S))
    np.testing.assert_allclose(np.abs(Kp * h), ref, rtol=1e-12)


def test_amplitude_distance_scaling_and_taper(orc):
    th = _theta()
    f = np.geomspace(1e-4, 1e-2, 50)
    h1, _, _ = orc.mode(th, 2, 2, f)
    h2, _, _ = orc.mode(_theta(D_L=2 * th[4]), 2, 2, f)
    np.testing.assert_allclose(h2, h1 / 2, rtol=1e-15, atol=0)
    M = th[0] * MSUN_S
    fcut = 6 ** -1.5 / math.pi / M
    assert np.all(h1[f >= fcut] == 0)
    assert np.all(np.abs(h1[f < 0.9 * fcut]) > 0)


def test_newtonian_chirp_time(orc):
    """t_c - t_f -> 5 M / (256 eta v^8) as v -> 0; the first corrections are the
    published 1PN and 1.5PN chirp-time terms (non-spinning)."""
    th = _theta(t_c=0.0, chi1=0.0, chi2=0.0)
    M = th[0] * MSUN_S
    eta = th[1] / (1 + th[1]) ** 2
    f = np.array([1e-7, 1e-6])
    _, _, tf = orc.mode(th, 2, 2, f)
    v = (math.pi * M * f) ** (1 / 3)
    tau0 = 5 * M / (256 * eta * v ** 8)
    dev = -tf / tau0 - 1
    # tau = tau0 (1 + (4/3)(743/336 + 11 eta/4) v^2 - (32 pi/5) v^3 + O(v^4))
    c2 = (4 / 3) * (743 / 336 + 11 * eta / 4)
    c3 = -32 * math.pi / 5
    resid = dev - (c2 * v ** 2 + c3 * v ** 3)
    assert np.all(np.abs(resid) < 100 * v ** 4)
    assert np.all(np.abs(dev) > 1e-4)
