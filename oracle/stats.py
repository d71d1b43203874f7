"""Statistics helpers for oracle validation (test infrastructure).

- ``tau_int``: integrated autocorrelation time with Sokal's automatic window
  (Sokal, "Monte Carlo methods in statistical mechanics", 1996 lectures):
  tau(W) = 1/2 + sum_{t=1..W} rho(t), W the first lag with W >= c * tau(W).
- ``binned_mean``: mean and standard error from non-overlapping bins.
- ``chi2_gof``: Pearson chi-square goodness of fit with pooling of cells whose
  expected count is below a floor.
"""
import numpy as np
from scipy import stats as _st


def autocorr(x):
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    y = x - x.mean()
    f = np.fft.rfft(y, n=2 * n)
    acf = np.fft.irfft(f * np.conj(f))[:n]
    acf /= np.arange(n, 0, -1)
    if acf[0] == 0:
        return np.zeros(n)
    return acf / acf[0]


def tau_int(x, c=6.0):
    rho = autocorr(x)
    tau = 0.5
    for w in range(1, len(rho)):
        tau += rho[w]
        if w >= c * tau:
            return float(tau), w
    return float(tau), len(rho) - 1


def binned_mean(x, nbins=32):
    x = np.asarray(x, dtype=np.float64)
    m = len(x) // nbins
    b = x[: m * nbins].reshape(nbins, m).mean(axis=1)
    return float(b.mean()), float(b.std(ddof=1) / np.sqrt(nbins))


def chi2_gof(observed, expected, min_expected=5.0):
    """Return (chi2, dof, p) after pooling all cells with expected < min_expected."""
    o = np.asarray(observed, dtype=np.float64)
    e = np.asarray(expected, dtype=np.float64)
    small = e < min_expected
    oo = list(o[~small])
    ee = list(e[~small])
    if small.any():
        oo.append(o[small].sum())
        ee.append(e[small].sum())
    oo = np.array(oo)
    ee = np.array(ee)
    chi2 = float(((oo - ee) ** 2 / ee).sum())
    dof = len(ee) - 1
    return chi2, dof, float(_st.chi2.sf(chi2, dof))
