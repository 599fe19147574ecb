"""Pins of the oracle's detector response (CPU only).

Each check is independent of the oracle's own formulas: a time-domain
brute-force evaluation with explicit delays, a closed-form limit, an algebraic
identity, a quadrature, or a published closed form.
"""
import math

import numpy as np
import pytest

from paper_2602_12011_amd import workloads as W

C_LIGHT = 299792458.0
AU = 149597870700.0


def _frame(rng):
    """A static equilateral triangle of side L (light-s) and a plane wave."""
    L = 8.339
    # random rotation
    A = np.linalg.qr(rng.normal(size=(3, 3)))[0]
    base = np.array([[0.0, 0.0, 0.0], [L, 0.0, 0.0], [L / 2, L * math.sqrt(3) / 2, 0.0]])
    base -= base.mean(axis=0)
    x = base @ A.T + rng.normal(scale=3.0, size=3)
    k = rng.normal(size=3)
    k /= np.linalg.norm(k)
    p = np.cross(k, rng.normal(size=3))
    p /= np.linalg.norm(p)
    q = np.cross(k, p)
    ep = np.outer(p, p) - np.outer(q, q)
    ec = np.outer(p, q) + np.outer(q, p)
    Hp = complex(rng.normal(), rng.normal())
    Hc = complex(rng.normal(), rng.normal())
    return L, x, k, ep, ec, Hp * ep + Hc * ec, Hp, Hc


def _td_link(f0, L, x, k, H, r, s, t):
    """Eq. (eq_td_resp) for h(t) = 2 Re[H e^{2 pi i f0 t}], evaluated in the time domain."""
    n = (x[r] - x[s]) / L

    def h_nn(tt):
        return 2.0 * np.real((n @ H @ n) * np.exp(2j * math.pi * f0 * tt))

    return (h_nn(t - L - k @ x[s]) - h_nn(t - k @ x[r])) / (2.0 * (1.0 - k @ n))


# Delay chains of eq. (eq_td_TDI) for X; each entry is (sign, link (r, s), number
# of one-arm delays).  With a rigid static triangle every delay operator is a
# shift by L.
_X15 = [(+1, (1, 3), 0), (+1, (3, 1), 1), (+1, (1, 2), 2), (+1, (2, 1), 3),
        (-1, (1, 2), 0), (-1, (2, 1), 1), (-1, (1, 3), 2), (-1, (3, 1), 3)]
_X20 = _X15 + [(+1, (1, 2), 4), (+1, (2, 1), 5), (+1, (1, 3), 6), (+1, (3, 1), 7),
               (-1, (1, 3), 4), (-1, (3, 1), 5), (-1, (1, 2), 6), (-1, (2, 1), 7)]


def _td_channel(chain, perm, f0, L, x, k, H, t):
    out = np.zeros_like(t)
    for sign, (r, s), nd in chain:
        rr, ss = perm[r] - 1, perm[s] - 1
        out += sign * _td_link(f0, L, x, k, H, rr, ss, t - nd * L)
    return out


def _project(sig, f0, t):
    return np.mean(sig * np.exp(-2j * math.pi * f0 * t))


@pytest.mark.parametrize("gen", [15, 20])
@pytest.mark.parametrize("f0", [3e-3, 2.1e-2, 4.7e-2])
def test_fd_links_and_tdi_match_time_domain_bruteforce(orc, gen, f0):
    rng = np.random.default_rng(int(f0 * 1e6) + gen)
    L, x, k, ep, ec, H, _, _ = _frame(rng)
    t = np.arange(64) / (64 * f0)          # one full cycle: projection is exact
    y_fd = orc.link_fd(f0, L, k, x, H)
    for r in range(3):
        for s in range(3):
            if r == s:
                continue
            y_td = _project(_td_link(f0, L, x, k, H, r, s, t), f0, t)
            assert abs(y_td - y_fd[r, s]) <= 1e-12 * np.abs(y_fd).max()
    xyz_fd, aet_fd = orc.tdi(f0, L, gen, y_fd)
    chain = _X15 if gen == 15 else _X20
    perms = [{1: 1, 2: 2, 3: 3}, {1: 2, 2: 3, 3: 1}, {1: 3, 2: 1, 3: 2}]
    xyz_td = np.array([_project(_td_channel(chain, p, f0, L, x, k, H, t), f0, t) for p in perms])
    scale = np.abs(xyz_fd).max()
    assert np.abs(xyz_td - xyz_fd).max() <= 1e-11 * scale
    X, Y, Z = xyz_td
    aet_td = np.array([(Z - X) / math.sqrt(2), (X - 2 * Y + Z) / math.sqrt(6),
                       (X + Y + Z) / math.sqrt(3)])
    assert np.abs(aet_td - aet_fd).max() <= 1e-11 * scale


def test_unit_separation_links(orc):
    """The link directions of exact Kepler orbits (unit = True: the unit
    separations, the transfer function keeping the nominal L).  On a triangle of
    side L they are the rigid triangle's (x_r - x_s) / L, so both options agree
    for any wave; with the wave travelling along the triangle's normal, k.n = 0
    and k.x_r = k.c for every spacecraft, so the unit-separation links do not
    change when the triangle is scaled about its centroid (with (x_r - x_s) / L
    they would scale as s^2)."""
    rng = np.random.default_rng(5)
    L, x, k, ep, ec, H, Hp, Hc = _frame(rng)
    for f in (3e-3, 2.1e-2):
        a, b = orc.link_fd(f, L, k, x, H), orc.link_fd(f, L, k, x, H, unit=True)
        assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()
    c = x.mean(axis=0)
    nrm = np.cross(x[1] - x[0], x[2] - x[0])
    kn = nrm / np.linalg.norm(nrm)
    p = np.cross(kn, rng.normal(size=3))
    p /= np.linalg.norm(p)
    q = np.cross(kn, p)
    Hn = Hp * (np.outer(p, p) - np.outer(q, q)) + Hc * (np.outer(p, q) + np.outer(q, p))
    for f in (3e-3, 2.1e-2):
        ref = orc.link_fd(f, L, kn, x, Hn, unit=True)
        for sc in (0.9, 1.03):
            xs = c + sc * (x - c)
            got = orc.link_fd(f, L, kn, xs, Hn, unit=True)
            assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), (f, sc)
            rigid = orc.link_fd(f, L, kn, xs, Hn)
            assert np.allclose(rigid[0, 1], sc ** 2 * ref[0, 1], rtol=1e-12)


def test_long_wavelength_limit_matches_antenna_pattern(orc):
    """fL << 1: X_1.5 -> 4 (2 pi f L)^2 (F+ h+ + Fx hx) e^{-2 pi i f k.x1}, with the
    60-degree Michelson pattern F = (b.e.b - a.e.a)/2 of the arms a, b leaving S/C 1."""
    rng = np.random.default_rng(7)
    L, x, k, ep, ec, H, Hp, Hc = _frame(rng)
    a = (x[1] - x[0]) / L
    b = (x[2] - x[0]) / L
    Fp = 0.5 * (b @ ep @ b - a @ ep @ a)
    Fc = 0.5 * (b @ ec @ b - a @ ec @ a)
    devs = []
    for f in (1e-6, 1e-5, 1e-4):
        y = orc.link_fd(f, L, k, x, H)
        xyz, _ = orc.tdi(f, L, 15, y)
        eps = 2 * math.pi * f * L
        X_lw = 4 * eps ** 2 * (Fp * Hp + Fc * Hc) * np.exp(-2j * math.pi * f * (k @ x[0]))
        devs.append(abs(xyz[0] / X_lw - 1))
    assert devs[0] < 1e-3
    # the deviation is O(f L): one decade in f is one decade in the deviation
    for d1, d2 in zip(devs, devs[1:]):
        assert 5 < d2 / d1 < 20


def test_t_channel_suppression_slope(orc):
    """|T|/|A| ~ (f L)^3 at low frequency."""
    rng = np.random.default_rng(11)
    L, x, k, ep, ec, H, _, _ = _frame(rng)
    ratio = []
    fs = np.array([1e-5, 1e-4])
    for f in fs:
        _, aet = orc.tdi(f, L, 20, orc.link_fd(f, L, k, x, H))
        ratio.append(abs(aet[2]) / abs(aet[0]))
    slope = np.log10(ratio[1] / ratio[0])
    assert 2.95 < slope < 3.05


def test_tdi_identities(orc):
    rng = np.random.default_rng(3)
    L, x, k, ep, ec, H, _, _ = _frame(rng)
    for f in (2e-4, 7e-3, 3.1e-2):
        y = orc.link_fd(f, L, k, x, H)
        x15, a15 = orc.tdi(f, L, 15, y)
        x20, a20 = orc.tdi(f, L, 20, y)
        z = np.exp(-2j * math.pi * f * L)
        assert np.allclose(x20, x15 * (1 - z ** 4), rtol=1e-12, atol=1e-14 * np.abs(x20).max())
        # A, E, T is an orthonormal rotation of X, Y, Z
        for xyz, aet in ((x15, a15), (x20, a20)):
            assert math.isclose(np.sum(np.abs(aet) ** 2), np.sum(np.abs(xyz) ** 2), rel_tol=1e-12)


@pytest.mark.parametrize("lm", W.MODES_HM)
def test_polarization_coefficients_from_time_domain_modes(orc, lm):
    """h_+ - i h_x = sum_{l,+-m} h_lm Y_lm with h_{l,-m} = (-1)^l conj(h_lm): the
    positive-frequency content of h_+, h_x is K+ h_{l,-m}, Kx h_{l,-m}."""
    l, m = lm
    iota = 0.7
    a = 0.3 - 0.8j
    om = 2 * math.pi * 1e-3
    t = np.arange(128) / 128 * (2 * math.pi / om)   # one orbital period
    h_pos = a * np.exp(-1j * m * om * t)                  # h_{l,m}
    h_neg = (-1) ** l * np.conj(a) * np.exp(1j * m * om * t)  # h_{l,-m}
    S = h_pos * orc.ylm(l, m, iota) + h_neg * orc.ylm(l, -m, iota)
    hp, hc = S.real, -S.imag
    f = m * om / (2 * math.pi)
    Kp, Kc = orc.pol_coeffs(l, m, iota)
    amp = (-1) ** l * np.conj(a)
    assert abs(_project(hp, f, t) - Kp * amp) < 1e-14
    assert abs(_project(hc, f, t) - Kc * amp) < 1e-14


def test_ylm_closed_forms_and_orthonormality(orc):
    for iota in (0.0, 0.4, 1.3, 2.9):
        c, s = math.cos(iota), math.sin(iota)
        assert math.isclose(orc.ylm(2, 2, iota), math.sqrt(5 / (64 * math.pi)) * (1 + c) ** 2,
                            rel_tol=1e-13, abs_tol=1e-16)
        assert math.isclose(orc.ylm(2, -2, iota), math.sqrt(5 / (64 * math.pi)) * (1 - c) ** 2,
                            rel_tol=1e-13, abs_tol=1e-16)
        assert math.isclose(orc.ylm(2, 1, iota), math.sqrt(5 / (16 * math.pi)) * s * (1 + c),
                            rel_tol=1e-13, abs_tol=1e-16)
        assert math.isclose(orc.ylm(2, -1, iota), math.sqrt(5 / (16 * math.pi)) * s * (1 - c),
                            rel_tol=1e-13, abs_tol=1e-16)
    # Gauss-Legendre quadrature over cos(iota), exact for these polynomials
    xg, wg = np.polynomial.legendre.leggauss(40)
    th = np.arccos(xg)
    Y = {(l, mm): np.array([orc.ylm(l, mm, v) for v in th])
         for (l, m) in W.MODES_HM for mm in (m, -m)}
    for key, y in Y.items():
        assert math.isclose(2 * math.pi * np.sum(wg * y * y), 1.0, rel_tol=1e-12)
    for m in (2, -2):
        assert abs(2 * math.pi * np.sum(wg * Y[(2, m)] * Y[(3, m)])) < 1e-13


@pytest.mark.parametrize("det", [W.LISA, W.TAIJI, W.TIANQIN], ids=lambda d: d["kind"])
def test_orbits_rigid_equilateral(orc, det):
    L = det["arm_m"] / C_LIGHT
    tol = 1e-13 if det["kind"] == "tianqin" else 1e-14
    for t in (0.0, 3.3e6, 1.7e7, 4.1e7):
        x = orc.orbit(det, t)
        for i, j in ((0, 1), (1, 2), (2, 0)):
            assert abs(np.linalg.norm(x[i] - x[j]) / L - 1) < tol
        centre = x.mean(axis=0)
        assert abs(np.linalg.norm(centre) * C_LIGHT / AU - 1) < 1e-12
        nrm = np.cross(x[1] - x[0], x[2] - x[0])
        nrm /= np.linalg.norm(nrm)
        if det["kind"] == "tianqin":
            lon, lat = det["tq_lon"], det["tq_lat"]
            nh = np.array([math.cos(lat) * math.cos(lon), math.cos(lat) * math.sin(lon), math.sin(lat)])
            assert abs(abs(nrm @ nh) - 1) < 1e-10
        else:
            # heliocentric: plane tilted 60 degrees to the ecliptic
            assert abs(abs(nrm[2]) - 0.5) < 1e-12
    # periods
    if det["kind"] == "tianqin":
        P = det["tq_period_s"]
        x0, x1 = orc.orbit(det, 1e5), orc.orbit(det, 1e5 + P)
        assert np.abs((x1 - x1.mean(0)) - (x0 - x0.mean(0))).max() < 1e-9
    else:
        x0, x1 = orc.orbit(det, 1e5), orc.orbit(det, 1e5 + W.YEAR_S)
        assert np.abs(x1 - x0).max() < 1e-9
        # revolution phase of the guiding centre
        xc = orc.orbit(det, 0.0).mean(axis=0)
        assert abs(math.atan2(xc[1], xc[0]) - det["phase0"]) < 1e-12


@pytest.mark.parametrize("det", [W.LISA, W.TAIJI, W.TIANQIN], ids=lambda d: d["kind"])
@pytest.mark.parametrize("gen", [15, 20])
def test_psd_matches_published_closed_forms(orc, det, gen):
    """S_X = 16 sin^2 x [S_oms + (3 + cos 2x) S_acc], S_XY = -8 sin^2 x cos x (S_oms + 4 S_acc),
    S_A = S_E = S_X - S_XY, S_T = S_X + 2 S_XY; TDI-2.0 multiplies by 4 sin^2 2x.
    S_T is compared with its cancellation-free form
    16 sin^2 x (1 - cos x) S_oms + 128 sin^2 x sin^4(x/2) S_acc."""
    d = dict(det, tdi_gen=gen)
    f = np.geomspace(1e-4, 3.3e-2, 97)
    SA, SE, ST = orc.psd(d, f)
    L = det["arm_m"] / C_LIGHT
    x = 2 * math.pi * f * L
    Soms = det["oms_asd"] ** 2 * (1 + (2e-3 / f) ** 4) * (2 * math.pi * f / C_LIGHT) ** 2
    Sacc = (det["acc_asd"] ** 2 * (1 + (4e-4 / f) ** 2) * (1 + (f / 8e-3) ** 4)
            / (2 * math.pi * f * C_LIGHT) ** 2)
    SX = 16 * np.sin(x) ** 2 * (Soms + (3 + np.cos(2 * x)) * Sacc)
    SXY = -8 * np.sin(x) ** 2 * np.cos(x) * (Soms + 4 * Sacc)
    fac = 4 * np.sin(2 * x) ** 2 if gen == 20 else 1.0
    # The oracle multiplies out the literal 1 - z^2 - z^4 + z^6, which cancels as
    # (2 pi f L)^2: about 1e-10 relative for TianQin's short arm at 0.1 mHz.
    rtol = 1e-9 if det["kind"] == "tianqin" else 1e-11
    np.testing.assert_allclose(SA, (SX - SXY) * fac, rtol=rtol)
    np.testing.assert_allclose(SE, (SX - SXY) * fac, rtol=rtol)
    ST_ref = (16 * np.sin(x) ** 2 * 2 * np.sin(x / 2) ** 2 * Soms
              + 128 * np.sin(x) ** 2 * np.sin(x / 2) ** 4 * Sacc)
    np.testing.assert_allclose(ST_ref, SX + 2 * SXY, rtol=1e-6)
    # the oracle forms T = (X + Y + Z)/sqrt3, which cancels as x^2 at low f
    np.testing.assert_allclose(ST, ST_ref * fac, rtol=1e-8)
