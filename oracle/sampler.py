"""TEST INFRASTRUCTURE ONLY -- plain reference of the ensemble sampler.

Counter-based random numbers (Philox4x32-10, Salmon et al., SC'11, written
from its published definition), the differential-evolution proposal over the
other half of the ensemble (ter Braak 2006), the box prior and
Metropolis-Hastings acceptance, in plain per-walker loops.  The likelihood is
any callable theta[B, 11] -> log L[B] (the oracle's, or an analytic target).
Shares no code with the GPU library.
"""
import math

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF

PURPOSE_PAIR, PURPOSE_GAMMA, PURPOSE_JITTER0, PURPOSE_ACCEPT = 0, 1, 2, 16
PURPOSE_MIX, PURPOSE_LATENT0 = 19, 20


def philox4x32_10(ctr, key):
    """One Philox4x32-10 block: ctr = 4 words, key = 2 words (python ints)."""
    c0, c1, c2, c3 = ctr
    k0, k1 = key
    for _ in range(10):
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = (p0 >> 32) & MASK, p0 & MASK
        hi1, lo1 = (p1 >> 32) & MASK, p1 & MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + W0) & MASK
        k1 = (k1 + W1) & MASK
    return c0, c1, c2, c3


def u01(a, b):
    """(0, 1) from two 32-bit words: 52 bits plus one half (max 1 - 2^-53)."""
    m = ((a << 20) ^ (b >> 12)) & ((1 << 52) - 1)
    return (m + 0.5) / 4503599627370496.0


def draw(seed, walker, step, purpose):
    return philox4x32_10((walker & MASK, step & MASK, (step >> 32) & MASK, purpose),
                         (seed & MASK, (seed >> 32) & MASK))


def log_prior(th, prior):
    lp = 0.0
    for j, (kind, lo, hi) in enumerate(prior):
        x = th[j]
        if kind == "uniform":
            if not (lo <= x <= hi):
                return -math.inf
        elif kind == "loguniform":
            if not (lo <= x <= hi):
                return -math.inf
            lp -= math.log(x)
        elif kind in ("cosine_sin", "sin"):
            if not (lo < x < hi):
                return -math.inf
            lp += math.log(math.sin(x))
        elif kind in ("arcsin", "cos"):
            if not (lo < x < hi):
                return -math.inf
            lp += math.log(math.cos(x))
        else:  # periodic, fixed
            if not math.isfinite(x):
                return -math.inf
    return lp


class DESampler:
    """Half-ensemble DE-MC: each step updates walkers [0, H) against [H, B),
    then [H, B) against [0, H).  With a flow (oracle.flow parameters, mu,
    sigma, p_flow) every updated walker takes, with probability p_flow, the
    flow's independence proposal instead (Metropolis-Hastings term
    log q(current) - log q(proposal))."""

    def __init__(self, loglike, prior, theta0, seed, tie_tol=1e-7, flow=None, tau=1.0):
        """tie_tol: |log u - Delta| below which an acceptance counts as a near tie
        (a decision another implementation could take the other way)."""
        self.flow = flow
        self.tau = tau
        self.loglike = loglike
        self.tie_tol = tie_tol
        self.prior = prior
        self.theta = np.array(theta0, dtype=np.float64)
        self.B = self.theta.shape[0]
        self.H0 = self.B // 2
        self.seed = seed
        self.step_no = 0
        free = [p for p in prior if p[0] != "fixed"]
        self.gamma = 2.38 / math.sqrt(2.0 * len(free))
        self.width = np.array([0.0 if p[0] == "fixed" else p[2] - p[1] for p in prior])
        self.logl = np.asarray(loglike(self.theta), dtype=np.float64)
        self.logp = np.array([log_prior(t, prior) for t in self.theta])
        self.accepts = np.zeros(self.B, dtype=np.int64)
        self.near_ties = 0

    def _propose(self, half):
        B, H0 = self.B, self.H0
        upd = range(H0, B) if half else range(0, H0)
        ref0, n_ref = (0, H0) if half else (H0, B - H0)
        step = self.step_no * 2 + half
        props = []
        for i in upd:
            r = draw(self.seed, i, step, PURPOSE_PAIR)
            r1 = min(int(u01(r[0], r[1]) * n_ref), n_ref - 1)
            r2 = min(int(u01(r[2], r[3]) * (n_ref - 1)), n_ref - 2)
            if r2 >= r1:
                r2 += 1
            g = draw(self.seed, i, step, PURPOSE_GAMMA)
            gamma = 1.0 if u01(g[0], g[1]) < 0.1 else self.gamma
            x = self.theta[i].copy()
            for k, (kind, lo, hi) in enumerate(self.prior):
                if kind == "fixed":
                    continue
                z4 = draw(self.seed, i, step, PURPOSE_JITTER0 + k)
                u1, u2 = u01(z4[0], z4[1]), u01(z4[2], z4[3])
                z = math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)
                xk = x[k] + gamma * (self.theta[ref0 + r1, k] - self.theta[ref0 + r2, k])
                xk = xk + 1e-6 * self.width[k] * z
                if kind == "periodic":
                    xk = lo + math.fmod(xk - lo, hi - lo)
                    if xk < lo:
                        xk += hi - lo
                x[k] = xk
            props.append(x)
        props = np.array(props)
        qratio = np.zeros(len(props))
        if self.flow is not None:
            props, qratio = self._flow_mix(list(upd), step, props, qratio)
        return list(upd), props, qratio

    def _flow_mix(self, upd, step, props, qratio):
        from oracle import flow as F
        flat, mu, sigma, p_flow = self.flow
        take, zs = [], []
        for j, i in enumerate(upd):
            r = draw(self.seed, i, step, PURPOSE_MIX)
            if u01(r[0], r[1]) < p_flow:
                z = []
                for k in range(11):
                    w = draw(self.seed, i, step, PURPOSE_LATENT0 + k)
                    u1, u2 = u01(w[0], w[1]), u01(w[2], w[3])
                    z.append(math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2))
                take.append(j)
                zs.append(z)
        self.last_latent = (np.array(take, dtype=np.int64), np.array(zs).reshape(-1, 11))
        if not take:
            return props, qratio
        take = np.array(take)
        # the latent point tau z enters in FP32
        z32 = (self.tau * np.array(zs)).astype(np.float32).astype(np.float64)
        u, _ = F.inverse(flat, z32)
        fprop = F.unstandardize(u, mu, sigma)
        lq_prop = F.log_prob(flat, fprop, mu, sigma, tau=self.tau)
        lq_cur = F.log_prob(flat, self.theta[[upd[j] for j in take]], mu, sigma, tau=self.tau)
        props = props.copy()
        props[take] = fprop
        qratio = qratio.copy()
        qratio[take] = lq_cur - lq_prop
        for jj, j in enumerate(take):
            for k, (kind, lo, hi) in enumerate(self.prior):
                if kind == "periodic" and not (lo <= fprop[jj, k] < hi):
                    qratio[j] = -math.inf
        return props, qratio

    def step(self):
        for half in (0, 1):
            idx, props, qratio = self._propose(half)
            Lp = np.asarray(self.loglike(props), dtype=np.float64)
            for j, i in enumerate(idx):
                lp = log_prior(props[j], self.prior)
                delta = (Lp[j] + lp) - (self.logl[i] + self.logp[i]) + qratio[j]
                r = draw(self.seed, i, self.step_no * 2 + half, PURPOSE_ACCEPT)
                lu = math.log(u01(r[0], r[1]))
                if math.isfinite(delta) and abs(lu - delta) < self.tie_tol:
                    self.near_ties += 1
                if math.isfinite(lp) and Lp[j] > -math.inf and lu < delta:
                    self.theta[i] = props[j]
                    self.logl[i] = Lp[j]
                    self.logp[i] = lp
                    self.accepts[i] += 1
        self.step_no += 1
