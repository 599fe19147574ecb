"""Seeded synthetic workloads: detector set-ups, frequency grids, the injection
and the walker draws.

This module holds configuration and random numbers only -- none of the
method's arithmetic -- so that both the GPU path and the CPU oracle can be fed
the same inputs.  Detector and grid descriptions are plain dicts.

Parameter order of a sample theta (11 doubles):
    [M_tot (Msun, detector frame), q = m2/m1, chi1, chi2, D_L (Gpc), iota,
     phi_c, lambda, beta, psi, t_c (s from the orbit epoch)]
"""
import math

import numpy as np

YEAR_S = 31557600.0          # Julian year, the grid spacing 1/yr of the long workloads
DAY_S = 86400.0

PARAM_NAMES = ("M_tot", "q", "chi1", "chi2", "D_L", "iota", "phi_c",
               "lambda", "beta", "psi", "t_c")

MODES_22 = [(2, 2)]
MODES_HM = [(2, 2), (2, 1), (3, 3), (3, 2), (4, 4)]

# Detectors.  Revolution phases: the Earth (and TianQin) at 0 deg, LISA 20 deg
# ahead and Taiji 20 deg behind (Sec. 3.2 places the three constellations at
# -20, 0 and +20 deg).  Noise amplitudes: OMS 15 pm/rtHz, acceleration
# 3 fm/s^2/rtHz for all three.
LISA = dict(kind="lisa", arm_m=2.5e9, phase0=math.radians(20.0), tdi_gen=20,
            oms_asd=15e-12, acc_asd=3e-15)
TAIJI = dict(kind="taiji", arm_m=3.0e9, phase0=math.radians(-20.0), tdi_gen=20,
             oms_asd=15e-12, acc_asd=3e-15)
TIANQIN = dict(kind="tianqin", arm_m=1.7e8, phase0=0.0, tdi_gen=20,
               oms_asd=15e-12, acc_asd=3e-15, tq_period_s=3.65 * DAY_S,
               tq_lon=math.radians(120.4), tq_lat=math.radians(-4.7))

# Injection (noise-free data are generated at this point).
THETA0 = np.array([1.0e6, 0.5, 0.2, 0.1, 10.0, math.pi / 3, 0.3, 1.0, 0.2, 0.5,
                   0.5 * YEAR_S])


def mtot_from_chirp(mc, q):
    """Total mass from the chirp mass and q = m2/m1: M = Mc eta^(-3/5), eta = q/(1+q)^2."""
    eta = q / (1.0 + q) ** 2
    return mc * eta ** -0.6


# The paper's own parameter-estimation set-up (Sec. 3.2): a 655360-s series
# at 10-s cadence, its rfftfreq bins kept within [1e-4, 5e-2] Hz, and the
# injection of its Table tab_pe_res (chirp mass 1.256227e6 Msun with q = 0.6,
# chi1 0.75, chi2 0.62, D_L 56 Gpc, iota 0.4, phi 1.3, lambda 1.375,
# beta -1.2108, psi 2.659, t_c 524288 s).  The stand-in waveform replaces
# PhenomXAS/XHM, so posteriors are not comparable with the paper's.
PE_T = 655360.0
PE_DT = 10.0
THETA_PE = np.array([mtot_from_chirp(1.256227e6, 0.6), 0.6, 0.75, 0.62, 56.0, 0.4, 1.3, 1.375,
                     -1.2108, 2.659, 524288.0])


def grid_series(T, f_lo=1e-4, f_hi=5e-2, dt=PE_DT):
    """rfftfreq bins k / T of a series of duration T at cadence dt, kept within [f_lo, f_hi]."""
    n_t = int(round(T / dt))
    k0 = math.ceil(f_lo * T)
    k1 = min(math.floor(f_hi * T), n_t // 2)
    return dict(f0=k0 / T, df=1.0 / T, n_bins=int(k1 - k0 + 1))


def grid_linear(f_lo, f_hi, n):
    """n bins from f_lo to f_hi inclusive."""
    return dict(f0=float(f_lo), df=(float(f_hi) - float(f_lo)) / (n - 1), n_bins=int(n))


def grid_rfft(n, df=1.0 / YEAR_S, f_lo=1e-4):
    """n bins of an rfftfreq-style grid (f = k df) starting at the first bin >= f_lo."""
    k0 = math.ceil(f_lo / df)
    return dict(f0=k0 * df, df=df, n_bins=int(n))


def config(name, n_bins=None):
    """Workload description by name.

    cfg0   one LISA-like detector, (2,2) only, 4096 bins over 1e-4..3e-2 Hz,
           1000 walkers (the small case the oracle runs in full);
    cfg1   one LISA-like detector, five modes, 2^20 bins at df = 1/yr, 4096 walkers;
    cfg2   LISA + Taiji + TianQin, five modes, 2^20 bins, 16384 walkers;
    cfg3   cfg1's signal, 1024 walkers for gradients, 256 for Fisher matrices;
    cfg4   cfg2's network and grid, 16384 walkers, with the learned proposal
           (11-D flow, 8 coupling layers of width 256);
    pe22, pehm, penet   the paper's three PE scenarios on its 32703-bin grid
           (LISA with (2,2) only; LISA with five modes; the three-detector
           network with five modes), injection THETA_PE.
    ``n_bins`` shortens the grid (same start and spacing) for quick tests.
    """
    if name == "cfg0":
        g = grid_linear(1e-4, 3e-2, 4096)
        c = dict(detectors=[LISA], modes=MODES_22, walkers=1000, **g)
    elif name == "cfg1":
        c = dict(detectors=[LISA], modes=MODES_HM, walkers=4096, **grid_rfft(1 << 20))
    elif name == "cfg2":
        c = dict(detectors=[LISA, TAIJI, TIANQIN], modes=MODES_HM, walkers=16384,
                 **grid_rfft(1 << 20))
    elif name == "cfg3":
        c = dict(detectors=[LISA], modes=MODES_HM, walkers=1024, fisher_points=256,
                 **grid_rfft(1 << 20))
    elif name == "cfg4":
        c = dict(detectors=[LISA, TAIJI, TIANQIN], modes=MODES_HM, walkers=16384,
                 flow=dict(layers=8, width=256), **grid_rfft(1 << 20))
    elif name in ("pe22", "pehm", "penet"):
        dets = [LISA, TAIJI, TIANQIN] if name == "penet" else [LISA]
        c = dict(detectors=dets, modes=MODES_22 if name == "pe22" else MODES_HM, walkers=1024,
                 **grid_series(PE_T))
    else:
        raise KeyError(name)
    c["name"] = name
    if n_bins is not None:
        c["n_bins"] = int(n_bins)
    return c


# Prior box of the walker draws.
PRIOR = dict(
    M_tot=("loguniform", 1e5, 1e7),
    q=("uniform", 0.1, 1.0),
    chi1=("uniform", -0.9, 0.9),
    chi2=("uniform", -0.9, 0.9),
    D_L=("loguniform", 1.0, 100.0),
    iota=("cosine_sin", 0.0, math.pi),      # arccos U[-1, 1]
    phi_c=("uniform", 0.0, 2 * math.pi),
    **{"lambda": ("uniform", 0.0, 2 * math.pi)},
    beta=("arcsin", -math.pi / 2, math.pi / 2),  # arcsin U[-1, 1]
    psi=("uniform", 0.0, math.pi),
    t_c=("uniform", THETA0[10] - 100.0, THETA0[10] + 100.0),
)

# Config 0 draws every coordinate uniformly over the same box.
PRIOR_FLAT = {k: ("uniform", v[1], v[2]) for k, v in PRIOR.items()}


def uniforms(n, seed, stream=0):
    """[n, 11] uniforms in [0, 1) from numpy's Philox4x32-10 bit generator."""
    bg = np.random.Philox(key=[int(seed) & 0xFFFFFFFFFFFFFFFF, int(stream)])
    return np.random.Generator(bg).random((n, 11))


def map_prior(u, prior=PRIOR):
    th = np.empty_like(u)
    for j, name in enumerate(PARAM_NAMES):
        kind, lo, hi = prior[name]
        x = u[:, j]
        if kind == "uniform":
            th[:, j] = lo + (hi - lo) * x
        elif kind == "loguniform":
            th[:, j] = np.exp(np.log(lo) + (np.log(hi) - np.log(lo)) * x)
        elif kind == "cosine_sin":
            th[:, j] = np.arccos(1.0 - 2.0 * x)
        elif kind == "arcsin":
            th[:, j] = np.arcsin(2.0 * x - 1.0)
        else:
            raise KeyError(kind)
    return th


def draw_walkers(n, seed=0x5EED, stream=0, flat=False):
    """n seeded samples from the prior box (flat=True: uniform in every coordinate)."""
    return map_prior(uniforms(n, seed, stream), PRIOR_FLAT if flat else PRIOR)


def prior_widths():
    """Scale of each coordinate (used to normalise derivative tolerances)."""
    return np.array([PRIOR[n][2] - PRIOR[n][1] for n in PARAM_NAMES])
