"""Pins of the oracle's exact Keplerian heliocentric orbits (orbit = 'kepler'):
what makes them Kepler ellipses of the stated elements is checked through
conserved quantities and limits, not by retyping the construction.

- two-body motion about the Sun with a = 1 AU and a 1-yr period: the specific
  energy v^2/2 - GM/r equals -GM/(2a) (vis-viva) and the angular momentum
  |r x v| equals sqrt(GM a (1 - e^2)) along the orbit, with GM = n^2 a^3 and
  the velocity from a fourth-order central difference of the positions;
- the orbital plane's inclination to the ecliptic: sin(i) = sqrt(3) e = L/(2 AU);
- periodicity over one year;
- the first-order limit: the exact ellipses approach the first-order
  triangle as e^2 (halving the arm divides the largest difference by four);
- the arms flex at order e^2 AU and at second order in L.
"""
import math

import numpy as np

from paper_2602_12011_amd import workloads as W

C_LIGHT = 299792458.0
AU = 149597870700.0
YR = 31557600.0


def _pos(orc, det, t):
    return orc.orbit(det, t) * C_LIGHT     # [3 spacecraft][3] in metres


def _vel(orc, det, t, h=2000.0):
    x = [_pos(orc, det, t + k * h) for k in (-2, -1, 1, 2)]
    return (x[0] - 8.0 * x[1] + 8.0 * x[2] - x[3]) / (12.0 * h)


def test_kepler_energy_angular_momentum_and_inclination(orc):
    for base in (W.LISA, W.TAIJI):
        det = dict(base, orbit="kepler")
        e = det["arm_m"] / (2.0 * math.sqrt(3.0) * AU)
        n = 2.0 * math.pi / YR
        GM = n * n * AU ** 3
        for t in np.linspace(0.0, YR, 13)[:-1] + 1234.5:
            x, v = _pos(orc, det, t), _vel(orc, det, t)
            for s in range(3):
                r = np.linalg.norm(x[s])
                energy = 0.5 * v[s] @ v[s] - GM / r
                assert abs(energy / (-GM / (2.0 * AU)) - 1.0) < 1e-9, (base["kind"], t, s)
                hvec = np.cross(x[s], v[s])
                hmag = np.linalg.norm(hvec)
                assert abs(hmag / math.sqrt(GM * AU * (1.0 - e * e)) - 1.0) < 1e-9
                sin_i = math.sqrt(hvec[0] ** 2 + hvec[1] ** 2) / hmag
                assert abs(sin_i - math.sqrt(3.0) * e) < 1e-9
                assert hvec[2] > 0.0                       # prograde, like the Earth


def test_kepler_periodic(orc):
    det = dict(W.LISA, orbit="kepler")
    for t in (0.0, 3.3e6, 2.0e7):
        assert np.abs(orc.orbit(det, t + YR) - orc.orbit(det, t)).max() < 1e-9


def test_kepler_first_order_limit_and_flexing(orc):
    worst, flex = [], []
    for arm in (2.5e9, 1.25e9):
        first = dict(W.LISA, arm_m=arm)
        kep = dict(first, orbit="kepler")
        e = arm / (2.0 * math.sqrt(3.0) * AU)
        e2R = e * e * AU / C_LIGHT                      # [light-s]
        dx, df = 0.0, 0.0
        for t in np.linspace(0.0, YR, 97):
            a, b = orc.orbit(first, t), orc.orbit(kep, t)
            dx = max(dx, float(np.abs(a - b).max()))
            for r, s in ((1, 2), (2, 0), (0, 1)):
                df = max(df, abs(np.linalg.norm(b[r] - b[s]) - arm / C_LIGHT))
                # the first-order triangle is exactly equilateral
                assert abs(np.linalg.norm(a[r] - a[s]) - arm / C_LIGHT) < 1e-12
        assert dx < 5.0 * e2R and df < 3.0 * e2R
        assert df > 0.3 * e2R                           # the exact arms do flex
        worst.append(dx)
        flex.append(df)
    assert 3.6 < worst[0] / worst[1] < 4.4, worst       # second order in e
    assert 3.6 < flex[0] / flex[1] < 4.4, flex


def test_kepler_injection_loglike_zero_and_small_change(orc):
    """On data made with the exact orbits log L(theta0) = 0, and the exact
    orbits move the response by a small, non-zero amount: the positions move
    by order e^2 AU (a phase of 2 pi f e^2 AU/c) and the arm directions turn by
    order e^2 AU / L."""
    cfg = W.config("cfg1", n_bins=6000)
    kep = dict(cfg, detectors=[dict(W.LISA, orbit="kepler")])
    d = orc.response(kep, W.THETA0)
    assert abs(orc.loglike(kep, d, W.THETA0)[0]) < 1e-9 * 0.5 * orc.inner(kep, d, d)
    h1 = orc.response(cfg, W.THETA0)
    rel = np.abs(d - h1).max() / np.abs(h1).max()
    f_top = cfg["f0"] + (cfg["n_bins"] - 1) * cfg["df"]
    e = W.LISA["arm_m"] / (2.0 * math.sqrt(3.0) * AU)
    e2R = e * e * AU / C_LIGHT
    assert 1e-9 < rel < 5.0 * e2R * (2.0 * math.pi * f_top + C_LIGHT / W.LISA["arm_m"])
