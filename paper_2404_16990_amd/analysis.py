"""Host-side analysis of observable traces (product code, not the oracle).

tau_int: integrated autocorrelation time of a scalar series with Sokal's
automatic window: rho(t) from the FFT autocovariance, tau(W) = 1/2 +
sum_{t=1..W} rho(t), W the first lag with W >= c * tau(W) (c = 6).
effective_rate: independent samples per second = units per second / (2 tau).
equilibration: automatic detection of the equilibrated part of a series
(Chodera, J. Chem. Theory Comput. 12, 1799 (2016)), the method the paper used
to discard non-equilibrated data: the start t0 that maximises the number of
effectively independent samples (n - t0) / g(t0), g = 1 + 2 sum_t rho(t) the
statistical inefficiency of x[t0:].
"""
import numpy as np


def autocorrelation(x):
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    d = x - x.mean()
    spec = np.fft.rfft(d, n=2 * n)
    cov = np.fft.irfft(spec * np.conj(spec))[:n] / np.arange(n, 0, -1)
    return cov / cov[0] if cov[0] > 0 else np.zeros(n)


def tau_int(x, c=6.0):
    """(tau, window); tau in units of the series' sampling interval."""
    rho = autocorrelation(x)
    tau = 0.5
    for w in range(1, rho.size):
        tau += rho[w]
        if w >= c * tau:
            return float(tau), w
    return float(tau), rho.size - 1


def effective_rate(units_per_second, tau):
    return units_per_second / (2.0 * tau)


def mean_and_error(x, tau):
    """Mean of a correlated series and its error sqrt(2 tau var / n); tau is
    floored at 1/2 (uncorrelated), since a windowed estimate of a short or
    anti-correlated series can fall below it."""
    x = np.asarray(x, dtype=np.float64)
    if x.size < 2:
        return float(x.mean()), float("nan")
    return float(x.mean()), float(np.sqrt(2.0 * max(tau, 0.5) * x.var(ddof=1) / x.size))


def statistical_inefficiency(x):
    """g = 1 + 2 sum_{t>=1} (1 - t/n) rho(t), summed until rho first drops to
    or below zero (the estimator of Chodera's method); g >= 1."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    if n < 3 or x.var() == 0.0:
        return 1.0
    rho = autocorrelation(x)
    g = 1.0
    for t in range(1, n - 1):
        if rho[t] <= 0.0:
            break
        g += 2.0 * rho[t] * (1.0 - t / n)
    return max(1.0, float(g))


def equilibration(x, candidates=100):
    """(t0, g, n_eff): the equilibrated part is x[t0:], chosen among about
    `candidates` evenly spaced starts as the one with the largest
    n_eff = (n - t0) / g(t0).  Starts leave at least 10 samples."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    best = (0, 1.0, 0.0)
    step = max(1, (n - 10) // candidates)
    for t0 in range(0, max(1, n - 10), step):
        g = statistical_inefficiency(x[t0:])
        ne = (n - t0) / g
        if ne > best[2]:
            best = (t0, g, ne)
    return best


def batch_means_error(x, n_bins=10):
    """Mean of a correlated series and the standard error of the mean of n_bins
    consecutive equal bins (the tail beyond a whole number of bins dropped).
    Independent of any autocorrelation estimate; unbiased once a bin is much
    longer than the series' autocorrelation time."""
    x = np.asarray(x, dtype=np.float64)
    m = x.size // n_bins
    if m < 1 or n_bins < 2:
        return float(x.mean()), float("nan")
    b = x[:m * n_bins].reshape(n_bins, m).mean(axis=1)
    return float(x.mean()), float(b.std(ddof=1) / np.sqrt(n_bins))
