"""Exact results for the periodic 2D Ising model (test infrastructure).

Used to pin the oracle, never called by the GPU library.

- ``T_C``: Onsager's critical temperature, 2 / ln(1 + sqrt 2) in units of
  J/k_B (paper section 3.1 prints it as 2.269185).
- ``yang_m``: spontaneous magnetisation [1 - sinh(2J/T)^-4]^(1/8) below T_c,
  0 above (the formula the paper's section 3.1 compares |M| against).
- ``onsager_u``: infinite-lattice internal energy per spin,
  u = -J coth(2K) [1 + (2/pi)(2 tanh^2(2K) - 1) K1(kappa)],
  kappa = 2 sinh(2K) / cosh^2(2K), K1 the complete elliptic integral of the
  first kind, K = J/T.
- ``enumerate_torus``: every state of a small torus, its bond sum B and
  magnetisation M, by brute force.
- ``transfer_lnZ``: ln Z of an n x m torus by the row-to-row transfer matrix.
- ``kaufman_lnZ`` / ``kaufman_energy``: ln Z of the finite n x m torus in
  closed form (Kaufman 1949; Ferdinand and Fisher 1969) and the exact mean
  energy per spin from its beta derivative.
"""
import itertools
import math

import mpmath
import numpy as np
from scipy import special

T_C = 2.0 / math.log(1.0 + math.sqrt(2.0))


def yang_m(T, J=1.0):
    if T >= T_C * J:
        return 0.0
    s = math.sinh(2.0 * J / T)
    return (1.0 - s ** -4) ** 0.125


def onsager_u(T, J=1.0):
    """Energy per spin of the infinite lattice (units of J when J = 1)."""
    K = J / T
    if abs(T - T_C * J) < 1e-13:
        return -math.sqrt(2.0) * J
    kappa = 2.0 * math.sinh(2 * K) / math.cosh(2 * K) ** 2
    k1 = special.ellipk(kappa * kappa)  # scipy's argument is the parameter m = kappa^2
    return -J / math.tanh(2 * K) * (1.0 + (2.0 / math.pi) * (2.0 * math.tanh(2 * K) ** 2 - 1.0) * k1)


def enumerate_torus(Lx, Ly):
    """(B, M) for every state of an Lx x Ly torus; state bit i <-> site i = y*Lx + x."""
    n = Lx * Ly
    assert n <= 20
    idx = np.arange(1 << n, dtype=np.int64)
    spins = 1 - 2 * ((idx[:, None] >> np.arange(n)) & 1)  # bit 1 -> -1, bit 0 -> +1
    s = spins.reshape(-1, Ly, Lx)
    B = (s * np.roll(s, -1, axis=2)).sum(axis=(1, 2)) + (s * np.roll(s, -1, axis=1)).sum(axis=(1, 2))
    M = s.sum(axis=(1, 2))
    return B.astype(np.int64), M.astype(np.int64)


def boltzmann_weights(B, T, J=1.0):
    """Normalised exp(beta J B) over an enumerated state list."""
    a = (J / T) * B.astype(np.float64)
    a -= a.max()
    w = np.exp(a)
    return w / w.sum()


def enum_moments(Lx, Ly, T, J=1.0):
    """Exact <e> (energy per spin / J) and <|m|> by enumeration."""
    B, M = enumerate_torus(Lx, Ly)
    p = boltzmann_weights(B, T, J)
    n = Lx * Ly
    return float(-(p * B).sum() / n), float((p * np.abs(M)).sum() / n)


def transfer_lnZ(n, m, K):
    """ln Z of a torus with rows of n spins and m rows, by the transfer matrix."""
    rows = np.array(list(itertools.product([1, -1], repeat=n)), dtype=np.float64)
    intra = (rows * np.roll(rows, -1, axis=1)).sum(axis=1)
    inter = rows @ rows.T
    # symmetric split of the intra-row bonds between the two rows a matrix joins
    Tm = np.exp(K * (0.5 * intra[:, None] + inter + 0.5 * intra[None, :]))
    ev = np.linalg.eigvalsh(Tm)
    top = ev.max()
    return float(m * math.log(top) + math.log(np.sum((ev / top) ** m)))


def _kaufman_lnZ_mp(n, m, K):
    """ln Z at the current mpmath precision (K an mpf)."""
    c2, s2 = mpmath.cosh(2 * K), mpmath.sinh(2 * K)
    base = c2 * c2 / s2  # cosh(2K) coth(2K)

    def gamma(l):
        if l == 0:
            return 2 * K + mpmath.log(mpmath.tanh(K))
        return mpmath.acosh(base - mpmath.cos(mpmath.pi * l / n))

    odd = [gamma(2 * r + 1) for r in range(n)]
    even = [gamma(2 * r) for r in range(n)]
    z1 = mpmath.fprod([2 * mpmath.cosh(m * g / 2) for g in odd])
    z2 = mpmath.fprod([2 * mpmath.sinh(m * g / 2) for g in odd])
    z3 = mpmath.fprod([2 * mpmath.cosh(m * g / 2) for g in even])
    z4 = mpmath.fprod([2 * mpmath.sinh(m * g / 2) for g in even])
    return mpmath.log(mpmath.mpf(0.5)) + (n * m / mpmath.mpf(2)) * mpmath.log(2 * s2) \
        + mpmath.log(z1 + z2 + z3 + z4)


def kaufman_lnZ(n, m, K, dps=60):
    """ln Z of the n x m periodic lattice at coupling K = beta*J (Kaufman's formula)."""
    with mpmath.workdps(dps):
        return _kaufman_lnZ_mp(n, m, mpmath.mpf(K))


def kaufman_energy(n, m, T, J=1.0, dps=60):
    """Exact <e> = <E>/(N J) of the n x m torus: -(1/N) d lnZ / dK."""
    with mpmath.workdps(dps):
        K = mpmath.mpf(J) / mpmath.mpf(T)
        d = mpmath.diff(lambda k: _kaufman_lnZ_mp(n, m, k), K)
        return float(-d / (n * m))
