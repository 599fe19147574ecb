"""Chain diagnostics for comparing proposals: integrated autocorrelation time
with Sokal's adaptive window, effective sample size, split-ensemble
Gelman-Rubin R-hat, and the two-sample Kolmogorov-Smirnov distance.  Host
code on numpy arrays of sampler output; no likelihood arithmetic."""
import numpy as np


def autocorr_function(x):
    """Normalized autocorrelation of a 1-D series (FFT, zero-padded)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    f = np.fft.rfft(x - x.mean(), n=2 * n)
    acf = np.fft.irfft(f * np.conj(f))[:n]
    return acf / acf[0] if acf[0] > 0 else np.zeros(n)


def _mean_autocorr(x):
    """Walker average of the normalized autocorrelation functions of the
    columns of x [T, walkers] (FFT along time, zero-padded); a constant walker
    contributes zeros."""
    T = x.shape[0]
    f = np.fft.rfft(x - x.mean(axis=0), n=2 * T, axis=0)
    acf = np.fft.irfft(f * np.conj(f), axis=0)[:T]
    a0 = acf[0]
    ok = a0 > 0
    rho = np.zeros(T)
    if ok.any():
        rho = (acf[:, ok] / a0[ok]).sum(axis=1)
    return rho / x.shape[1]


def integrated_time(chain, c=5.0):
    """tau of each parameter for chain [T, walkers, d]: the autocorrelation
    function averaged over walkers, summed up to the smallest window M with
    M >= c tau(M) (Sokal 1997)."""
    chain = np.asarray(chain, dtype=np.float64)
    T, B, d = chain.shape
    taus = np.empty(d)
    for j in range(d):
        rho = np.zeros(T)
        for b0 in range(0, B, 4096):
            rho += _mean_autocorr(chain[:, b0:b0 + 4096, j]) * min(4096, B - b0)
        rho /= B
        tau_m = 2.0 * np.cumsum(rho) - 1.0
        m = np.arange(T)
        ok = m >= c * tau_m
        w = int(np.argmax(ok)) if ok.any() else T - 1
        taus[j] = max(tau_m[w], 1.0)
    return taus


def ess(chain, c=5.0):
    """Effective sample size per parameter: walkers * T / tau."""
    chain = np.asarray(chain)
    T, B, _ = chain.shape
    return B * T / integrated_time(chain, c)


def gelman_rubin(chain, groups=4):
    """Split-ensemble R-hat per parameter: the walkers are split into `groups`
    equal sets, each set's pooled draws treated as one chain."""
    chain = np.asarray(chain, dtype=np.float64)
    T, B, d = chain.shape
    g = B // groups
    x = chain[:, :g * groups, :].reshape(T, groups, g, d).transpose(1, 0, 2, 3).reshape(groups, T * g, d)
    n = x.shape[1]
    means = x.mean(axis=1)
    W = x.var(axis=1, ddof=1).mean(axis=0)
    Bv = n * means.var(axis=0, ddof=1)
    var = (n - 1) / n * W + Bv / n
    return np.sqrt(var / W)


def ks_distance(a, b):
    """Two-sample Kolmogorov-Smirnov statistic of 1-D samples."""
    a = np.sort(np.asarray(a, dtype=np.float64))
    b = np.sort(np.asarray(b, dtype=np.float64))
    v = np.concatenate([a, b])
    ca = np.searchsorted(a, v, side="right") / a.size
    cb = np.searchsorted(b, v, side="right") / b.size
    return float(np.abs(ca - cb).max())
