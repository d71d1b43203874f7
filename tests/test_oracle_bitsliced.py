"""Pins of the bit-sliced random-number contract (rng = 1) beyond the
brute-force sweeps and the distribution tests that cover both contracts.

- The lazy comparison the GPU kernel performs (threshold and uniform compared
  most significant bit first, stopping at the first differing bit) equals the
  integer comparison u < thr: checked exhaustively on 8-bit values and on
  random 32-bit values, written here independently of both implementations.
- The transposed uniforms are uniform on [0, 2^32): 100-bin chi-square, the
  frequency of every bit, and the lag-1 joint histogram of neighbouring sites
  of a group (they share words, so this is where a dependence would show).
"""
import numpy as np
import pytest

import oracle
from oracle import philox, stats


def _lazy_less(u, thr, bits):
    """u < thr decided bit by bit from the top, as the GPU path does."""
    for k in range(bits - 1, -1, -1):
        ub, tb = (u >> k) & 1, (thr >> k) & 1
        if ub != tb:
            return ub < tb
    return False  # all bits equal: u == thr, not less


def test_lazy_comparison_exhaustive_8_bit():
    for u in range(256):
        for thr in range(256):
            assert _lazy_less(u, thr, 8) == (u < thr)


def test_lazy_comparison_random_32_bit():
    rng = np.random.default_rng(11)
    u = rng.integers(0, 2**32, size=20000, dtype=np.uint64)
    thr = rng.integers(0, 2**32, size=20000, dtype=np.uint64)
    thr[:2000] = u[:2000]  # ties
    thr[2000:4000] = u[2000:4000] ^ 1  # differ only in the last bit
    for a, b in zip(u.tolist(), thr.tolist()):
        assert _lazy_less(a, b, 32) == (a < b)


def _group_uniforms(seed, replica, t, colour, groups):
    """Transposed uniforms of whole groups, from the pure-Python Philox."""
    out = []
    key = philox.seed_key(seed)
    for g in range(groups):
        w = []
        for m in range(8):
            w.extend(philox.philox4x32_10((8 * g + m, t, replica, colour), key))
        for b in range(32):
            out.append(sum(((w[k] >> b) & 1) << (31 - k) for k in range(32)))
    return np.array(out, dtype=np.uint64)


def test_group_uniforms_equal_site_definition():
    # the site-by-site definition agrees with whole-group transposition
    Lx = 128
    u = _group_uniforms(5, 2, 3, 1, 2)
    for h in range(64):
        y, rem = divmod(2 * h, Lx)
        x = rem + ((1 + y) & 1)  # colour-1 site with compact index h
        assert philox.bitsliced_uniform(5, 2, 3, 1, Lx, x, y) == int(u[h])


def test_transposed_uniforms_are_uniform():
    u = _group_uniforms(2024, 7, 11, 0, 160)  # 5120 values
    u = np.concatenate([u, _group_uniforms(99, 1, 0, 1, 160)])
    counts = np.bincount((u * 100 >> 32).astype(np.int64), minlength=100)
    chi2, dof, p = stats.chi2_gof(counts, np.full(100, len(u) / 100))
    assert p > 1e-3, (chi2, p)
    bits = ((u[:, None] >> np.arange(32, dtype=np.uint64)) & 1).astype(np.float64)
    freq = bits.mean(axis=0)
    assert np.all(np.abs(freq - 0.5) < 5 * 0.5 / np.sqrt(len(u)))
    # neighbouring sites of a group: joint 10 x 10 histogram of (u_b, u_b+1)
    g = u.reshape(-1, 32)
    a, b = (g[:, :-1].ravel() * 10 >> 32), (g[:, 1:].ravel() * 10 >> 32)
    joint = np.bincount((a * 10 + b).astype(np.int64), minlength=100)
    chi2, dof, p = stats.chi2_gof(joint, np.full(100, a.size / 100))
    assert p > 1e-3, (chi2, p)


def test_contracts_differ_but_agree_in_distribution_of_first_sweep():
    # same seed, different contract: different trajectories, same initial state
    d0 = oracle.desc(64, 64, 1.0, 0.44, seed=3, replica=1, rng=0)
    d1 = oracle.desc(64, 64, 1.0, 0.44, seed=3, replica=1, rng=1)
    s0, s1 = oracle.init_state(d0), oracle.init_state(d1)
    assert np.array_equal(s0, s1)
    oracle.sweeps(d0, s0, 3)
    oracle.sweeps(d1, s1, 3)
    assert not np.array_equal(s0, s1)


def test_invalid_rng_rejected():
    d = oracle.desc(8, 8, 1.0, 0.4, rng=2)
    with pytest.raises(Exception):
        oracle.init_state(d)
