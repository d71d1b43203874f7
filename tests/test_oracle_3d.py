"""Pins of the 3D (simple cubic, six neighbours) oracle against what the
physics fixes independently of the oracle's code:

- beta = 0 (every proposal accepted: a sweep negates the state) and
  beta = infinity (a cold start is frozen; energy never rises) in closed form;
- sampled states against exhaustive enumeration of the Boltzmann law on the
  2x2x2 torus (all 256 states) and on the 4x2x2 torus ((B, M) classes);
- the high-temperature series of the nearest-neighbour correlation,
  <s s'> = t + 4 t^3 + O(t^5) with t = tanh(beta J) (each bond of the simple
  cubic lattice lies on 4 plaquettes; the square lattice's t + 2 t^3 is
  checked against Onsager as a control);
- the low-temperature series of the magnetisation of a cold start,
  m = 1 - 2 u^6 - 12 u^10 + O(u^12) with u = exp(-2 beta J) (one reversed
  spin breaks 6 bonds, two adjacent ones 10; 3 bond directions per site).
The distribution and series pins run under both random-number contracts
(rng = 0 one Philox word per site, rng = 1 bit-sliced group words).
Seeds are fixed, so pass/fail is deterministic.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import exact, stats


def _enumerate3(Lx, Ly, Lz):
    """(B, M, spins) of every state of a small periodic Lx x Ly x Lz lattice."""
    n = Lx * Ly * Lz
    idx = np.arange(1 << n, dtype=np.int64)
    s = (1 - 2 * ((idx[:, None] >> np.arange(n)) & 1)).reshape(-1, Lz, Ly, Lx)
    B = (s * (np.roll(s, -1, axis=3) + np.roll(s, -1, axis=2) + np.roll(s, -1, axis=1))).sum(axis=(1, 2, 3))
    return B, s.sum(axis=(1, 2, 3)), s


def test_thresholds_closed_form():
    for beta in (0.1, 0.2216546, 0.5):
        thr4, thr8, thr12, always = oracle.thresholds3(1.0, beta)
        for k, thr in ((1, thr4), (2, thr8), (3, thr12)):
            assert thr == math.floor(math.exp(-4 * k * beta) * 2 ** 32)
        assert always == 0
    assert oracle.thresholds3(1.0, 0.0)[3] == 1
    assert oracle.thresholds3(1.0, math.inf)[:3] == (0, 0, 0)


def test_beta_zero_negates_every_sweep():
    d = oracle.desc3(6, 4, 8, beta=0.0, seed=3)
    s = oracle.init_state3(d)
    s0 = s.copy()
    oracle.sweeps3(d, s, 1)
    np.testing.assert_array_equal(s, -s0)
    oracle.sweeps3(d, s, 1, t0=1)
    np.testing.assert_array_equal(s, s0)


def test_infinite_beta():
    d = oracle.desc3(6, 4, 4, beta=math.inf, seed=4, init=oracle.INIT_UP)
    s = oracle.init_state3(d)
    oracle.sweeps3(d, s, 5)
    assert (s == 1).all()
    d = oracle.desc3(8, 6, 4, beta=math.inf, seed=5)
    s = oracle.init_state3(d)
    b, _ = oracle.sweeps3(d, s, 30, record_every=1)
    assert np.all(np.diff(b) >= 0) and b[0] >= oracle.observables3(oracle.init_state3(d))[0]


def test_observables_match_definition():
    d = oracle.desc3(6, 4, 2, seed=9)
    s = oracle.init_state3(d)
    B = int((s * (np.roll(s, -1, 2) + np.roll(s, -1, 1) + np.roll(s, -1, 0))).sum())
    assert oracle.observables3(s) == (B, int(s.sum()))


def _zero_field(s):
    f = sum(np.roll(s, k, ax) for ax in (-1, -2, -3) for k in (1, -1))
    return (f == 0).all(axis=(-3, -2, -1))


@pytest.mark.parametrize("T,rng", [(2.0, 0), (4.5, 0), (8.0, 0), (2.0, 1), (4.5, 1)])
def test_2x2x2_states_chi2(T, rng):
    """Every site of the 2x2x2 torus has three distinct neighbours, each
    joined by two bonds, so no local field vanishes and the chain is ergodic."""
    R = 1 << 15
    descs = [oracle.desc3(2, 2, 2, beta=1.0 / T, seed=2020 + int(T * 10) + rng, replica=r, rng=rng) for r in range(R)]
    states = [oracle.init_state3(d) for d in descs]
    oracle.run_batch3(descs, states, 60)
    idx = np.array([int(((st.reshape(-1) < 0) * (1 << np.arange(8))).sum()) for st in states])
    B, _, _ = _enumerate3(2, 2, 2)
    p = np.exp((B - B.max()) / T)
    p /= p.sum()
    chi2, dof, pval = stats.chi2_gof(np.bincount(idx, minlength=256), R * p)
    assert pval > 1e-3, (chi2, dof, pval)


@pytest.mark.parametrize("T,rng", [(3.0, 0), (4.5, 0), (7.0, 0), (4.5, 1)])
def test_4x2x2_classes_chi2(T, rng):
    """(B, M) classes of the 4x2x2 torus; states in which every local field
    vanishes (a closed set for the checkerboard rule, which flips them without
    a draw) are excluded from both sides and their share bounded."""
    R = 1 << 15
    descs = [oracle.desc3(4, 2, 2, beta=1.0 / T, seed=4040 + int(T * 10) + rng, replica=r, rng=rng) for r in range(R)]
    states = [oracle.init_state3(d) for d in descs]
    oracle.run_batch3(descs, states, 80)
    arr = np.array(states)
    zf = _zero_field(arr)
    assert zf.mean() < 5e-3, zf.mean()
    arr = arr[~zf]
    Bs = (arr * (np.roll(arr, -1, 3) + np.roll(arr, -1, 2) + np.roll(arr, -1, 1))).sum(axis=(1, 2, 3))
    Ms = arr.sum(axis=(1, 2, 3))
    eB, eM, es = _enumerate3(4, 2, 2)
    p = np.exp((eB - eB.max()) / T)
    p[_zero_field(es)] = 0.0
    p /= p.sum()
    keys = (eB + 64) * 64 + (eM + 32)
    uk, inv = np.unique(keys, return_inverse=True)
    expected = np.bincount(inv, weights=p) * len(arr)
    ok = np.searchsorted(uk, (Bs + 64) * 64 + (Ms + 32))
    chi2, dof, pval = stats.chi2_gof(np.bincount(ok, minlength=uk.size), expected)
    assert pval > 1e-3, (chi2, dof, pval)


def test_square_lattice_series_control():
    """The counting behind the 3D series, on the square lattice: t + 2 t^3
    matches Onsager's exact energy to O(t^5)."""
    for T in (10.0, 12.0):
        t = math.tanh(1.0 / T)
        assert abs(-exact.onsager_u(T) / 2 - (t + 2 * t ** 3)) < 6 * t ** 5


@pytest.mark.parametrize("T,rng", [(10.0, 0), (12.0, 0), (12.0, 1)])
def test_high_temperature_series(T, rng):
    L, R, n = 24, 8, 1500
    descs = [oracle.desc3(L, L, L, beta=1.0 / T, seed=777 + int(T) + rng, replica=r, rng=rng) for r in range(R)]
    states = [oracle.init_state3(d) for d in descs]
    bond, _ = oracle.run_batch3(descs, states, n, record_every=1)
    ss = bond[:, 100:].astype(np.float64) / (3 * L ** 3)
    per_rep = ss.mean(axis=1)
    mean, err = per_rep.mean(), per_rep.std(ddof=1) / math.sqrt(R)
    t = math.tanh(1.0 / T)
    series = t + 4 * t ** 3
    assert abs(mean - series) < 40 * t ** 5 + 4 * err, (mean, series, err, t ** 5)
    # the t^3 term is resolved: the square-lattice coefficient would fail
    assert abs(mean - (t + 2 * t ** 3)) > 4 * err + 40 * t ** 5


@pytest.mark.parametrize("T,rng", [(1.8, 0), (2.0, 0), (2.0, 1)])
def test_low_temperature_magnetisation(T, rng):
    L, R, n = 24, 8, 1000
    descs = [oracle.desc3(L, L, L, beta=1.0 / T, seed=555 + int(10 * T) + rng, replica=r, init=oracle.INIT_UP,
                          rng=rng) for r in range(R)]
    states = [oracle.init_state3(d) for d in descs]
    _, mag = oracle.run_batch3(descs, states, n, record_every=1)
    m = mag[:, 50:].astype(np.float64) / L ** 3
    per_rep = m.mean(axis=1)
    mean, err = per_rep.mean(), per_rep.std(ddof=1) / math.sqrt(R)
    u = math.exp(-2.0 / T)
    series = 1 - 2 * u ** 6 - 12 * u ** 10
    assert abs(mean - series) < 20 * u ** 12 + 4 * err, (mean, series, err, u ** 12)


def test_contracts_agree_where_no_draw_is_made():
    """At beta = 0 and beta = infinity no proposal draws a uniform, so both
    random-number contracts give the same trajectory; at finite beta they
    differ."""
    for beta in (0.0, math.inf):
        a = oracle.desc3(64, 4, 6, beta=beta, seed=12, rng=0)
        b = oracle.desc3(64, 4, 6, beta=beta, seed=12, rng=1)
        sa, sb = oracle.init_state3(a), oracle.init_state3(b)
        oracle.sweeps3(a, sa, 5)
        oracle.sweeps3(b, sb, 5)
        np.testing.assert_array_equal(sa, sb)
    a = oracle.desc3(64, 4, 6, beta=0.3, seed=12, rng=0)
    b = oracle.desc3(64, 4, 6, beta=0.3, seed=12, rng=1)
    sa, sb = oracle.init_state3(a), oracle.init_state3(b)
    oracle.sweeps3(a, sa, 5)
    oracle.sweeps3(b, sb, 5)
    assert (sa != sb).any()
