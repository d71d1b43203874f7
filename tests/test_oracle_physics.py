"""Statistical pins: the oracle's trajectory samples the Boltzmann distribution.

- 4x4 torus: chi-square of sampled states against exhaustive enumeration.
- 16x16 and 32x32 at T_c: mean energy against Kaufman's exact finite torus.
- 128x128 away from T_c: mean energy against Onsager, <|m|> against Yang.
All seeds are fixed, so pass/fail is deterministic; thresholds are p > 1e-3
or |z| < 4 with errors from independent replicas.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import exact, stats


def _final_states(L, T, R, n_sweeps, seed0, rng=0):
    descs = [oracle.desc(L, L, 1.0, 1.0 / T, seed=seed0, replica=r, rng=rng) for r in range(R)]
    states = [oracle.init_state(d) for d in descs]
    oracle.run_batch(descs, states, n_sweeps)
    return states


def _zero_field(s):
    """True for states in which every site's four neighbours sum to zero."""
    f = np.roll(s, 1, -1) + np.roll(s, -1, -1) + np.roll(s, 1, -2) + np.roll(s, -1, -2)
    return (f == 0).all(axis=(-2, -1))


def _enumerated_zero_field(L):
    idx = np.arange(1 << (L * L), dtype=np.int64)
    spins = (1 - 2 * ((idx[:, None] >> np.arange(L * L)) & 1)).reshape(-1, L, L)
    return _zero_field(spins)


# The checkerboard rule flips every site with dE <= 0 without a draw.  In a
# state where every local field is zero (e.g. 2x2 blocks in a checkerboard on a
# torus whose sides are multiples of 4) every site of a colour flips, the other
# colour's fields stay zero, and the sweep maps the state to another such state:
# the set Z of zero-field states is closed and deterministic.  On the 4x4 torus
# a few random starts in 10^4 fall into it, so the sampled states are compared
# with the Boltzmann law outside Z, and the fraction caught in Z is bounded.

@pytest.mark.parametrize("T,rng", [(1.5, 0), (exact.T_C, 0), (3.0, 0), (5.0, 0), (1.5, 1), (exact.T_C, 1),
                                   (5.0, 1)])
def test_4x4_state_classes_chi2(T, rng):
    R = 1 << 16
    states = _final_states(4, T, R, 200, seed0=424242 + int(100 * T) + 7 * rng, rng=rng)
    zf = _zero_field(np.array(states).reshape(R, 4, 4))
    assert zf.mean() < 2e-3, zf.mean()
    states = [s for s, z in zip(states, zf) if not z]
    R = len(states)
    B = np.array([oracle.observables(s)[0] for s in states])
    M = np.array([int(s.sum()) for s in states])
    eB, eM = exact.enumerate_torus(4, 4)
    p = exact.boltzmann_weights(eB, T)
    p[_enumerated_zero_field(4)] = 0.0
    p /= p.sum()
    keys = (eB + 64) * 64 + (eM + 32)
    uk, inv = np.unique(keys, return_inverse=True)
    expected = np.bincount(inv, weights=p) * R
    obs_keys = (B + 64) * 64 + (M + 32)
    pos = np.searchsorted(uk, obs_keys)
    assert (uk[pos] == obs_keys).all()  # every sampled (B, M) is a reachable class
    observed = np.bincount(pos, minlength=len(uk))
    chi2, dof, pval = stats.chi2_gof(observed, expected)
    assert pval > 1e-3, (T, chi2, dof, pval)


def test_4x4_full_state_histogram_chi2():
    T = 5.0
    R = 1 << 17
    states = _final_states(4, T, R, 100, seed0=777)
    zf = _zero_field(np.array(states).reshape(R, 4, 4))
    assert zf.mean() < 2e-3, zf.mean()
    states = [s for s, z in zip(states, zf) if not z]
    R = len(states)
    bits = (np.array([s.ravel() for s in states]) < 0).astype(np.int64)
    idx = (bits << np.arange(16)).sum(axis=1)  # same state numbering as enumerate_torus
    eB, _ = exact.enumerate_torus(4, 4)
    p = exact.boltzmann_weights(eB, T)
    p[_enumerated_zero_field(4)] = 0.0
    expected = p / p.sum() * R
    observed = np.bincount(idx, minlength=1 << 16)
    chi2, dof, pval = stats.chi2_gof(observed, expected)
    assert pval > 1e-3, (chi2, dof, pval)


def _energy_runs(L, T, R, n_sweeps, burn, init, seed, rng=0):
    descs = [oracle.desc(L, L, 1.0, 1.0 / T, seed=seed + r, replica=r, init=init, rng=rng) for r in range(R)]
    states = [oracle.init_state(d) for d in descs]
    b, m = oracle.run_batch(descs, states, n_sweeps, record_every=1)
    N = L * L
    e = -b[:, burn:].astype(np.float64) / N
    am = np.abs(m[:, burn:]).astype(np.float64) / N
    return e, am


def _z(samples, target):
    means = samples.mean(axis=1)
    err = means.std(ddof=1) / math.sqrt(len(means))
    return (means.mean() - target) / err, means.mean(), err


@pytest.mark.parametrize("L,rng", [(16, 0), (32, 0), (16, 1), (64, 1)])
def test_kaufman_energy_at_tc(L, rng):
    e, _ = _energy_runs(L, exact.T_C, 48, 4000, 1000, oracle.INIT_RANDOM, seed=5000 + L, rng=rng)
    target = exact.kaufman_energy(L, L, exact.T_C)
    z, mean, err = _z(e, target)
    assert abs(z) < 4, (L, mean, target, err)
    assert err < 3e-3


@pytest.mark.parametrize("T", [1.5, 2.0, 3.0, 3.5])
def test_onsager_energy_and_yang_magnetisation_128(T):
    init = oracle.INIT_UP if T < exact.T_C else oracle.INIT_RANDOM
    e, am = _energy_runs(128, T, 16, 1200, 300, init, seed=9000 + int(10 * T))
    z, mean, err = _z(e, exact.onsager_u(T))
    assert abs(z) < 4, (T, mean, exact.onsager_u(T), err)
    if T < exact.T_C:
        z, mean, err = _z(am, exact.yang_m(T))
        assert abs(z) < 4, (T, mean, exact.yang_m(T), err)
    else:
        # above T_c, <|m|> ~ sqrt(chi T / N) -> small on 128^2
        assert am.mean() < 0.1


def test_wrong_rule_would_fail():
    """The 4x4 class test detects a plausible mistake: the three-neighbour sum
    printed in the FlipSpin listing gives a different stationary law.  Here a
    3-neighbour Metropolis chain is simulated in numpy and must fail the test."""
    rng = np.random.default_rng(3)
    T = exact.T_C
    R = 1 << 14
    s = np.where(rng.random((R, 4, 4)) < 0.5, 1, -1).astype(np.int64)
    y, x = np.indices((4, 4))
    for _ in range(60):
        for c in (0, 1):
            mask = ((x + y) & 1) == c
            nsum = np.roll(s, 1, 2) + np.roll(s, -1, 2) + np.roll(s, 1, 1)  # dropped term
            dE = 2 * s * nsum
            acc = (dE <= 0) | (rng.random(s.shape) < np.exp(-np.maximum(dE, 0) / T))
            s = np.where(mask & acc, -s, s)
    B = (s * np.roll(s, -1, 2)).sum(axis=(1, 2)) + (s * np.roll(s, -1, 1)).sum(axis=(1, 2))
    M = s.sum(axis=(1, 2))
    eB, eM = exact.enumerate_torus(4, 4)
    p = exact.boltzmann_weights(eB, T)
    keys = (eB + 64) * 64 + (eM + 32)
    uk, inv = np.unique(keys, return_inverse=True)
    expected = np.bincount(inv, weights=p) * R
    pos = np.searchsorted(uk, (B + 64) * 64 + (M + 32))
    observed = np.bincount(pos, minlength=len(uk))
    _, _, pval = stats.chi2_gof(observed, expected)
    assert pval < 1e-6
