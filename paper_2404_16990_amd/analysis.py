"""Host-side analysis of observable traces (product code, not the oracle).

tau_int: integrated autocorrelation time of a scalar series with Sokal's
automatic window: rho(t) from the FFT autocovariance, tau(W) = 1/2 +
sum_{t=1..W} rho(t), W the first lag with W >= c * tau(W) (c = 6).
effective_rate: independent samples per second = units per second / (2 tau).
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
    """Mean of a correlated series and its error sqrt(2 tau var / n)."""
    x = np.asarray(x, dtype=np.float64)
    return float(x.mean()), float(np.sqrt(2.0 * tau * x.var(ddof=1) / x.size))
