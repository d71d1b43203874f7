"""Pins for the oracle's random-number generator (Philox4x32-10).

The paper's generator is unpublished (Supplementary S.4), so the contract uses
Philox4x32-10.  Pins: the published known-answer vectors, agreement of the C
oracle with an independent pure-Python implementation, and the paper's own
uniformity checks (Supplementary S.4/S.5: 100-bin histogram, lag-1 joint
histogram, NIST SP 800-22 frequency / block-frequency / runs tests) applied to
the stream the contract feeds the sweep.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import special, stats

import oracle
from oracle import philox as pyphilox

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox_kat.json")


def _kat():
    with open(GOLDEN) as f:
        return json.load(f)["vectors"]


@pytest.mark.parametrize("vec", _kat())
def test_kat_c_oracle(vec):
    ctr = [int(v, 16) for v in vec["ctr"]]
    key = [int(v, 16) for v in vec["key"]]
    assert oracle.philox4x32_10(ctr, key) == [int(v, 16) for v in vec["out"]]


@pytest.mark.parametrize("vec", _kat())
def test_kat_python(vec):
    ctr = [int(v, 16) for v in vec["ctr"]]
    key = [int(v, 16) for v in vec["key"]]
    assert pyphilox.philox4x32_10(ctr, key) == [int(v, 16) for v in vec["out"]]


def test_c_matches_python_random_counters():
    rng = np.random.default_rng(7)
    for _ in range(500):
        ctr = [int(v) for v in rng.integers(0, 2**32, size=4, dtype=np.uint64)]
        key = [int(v) for v in rng.integers(0, 2**32, size=2, dtype=np.uint64)]
        assert oracle.philox4x32_10(ctr, key) == pyphilox.philox4x32_10(ctr, key)


def _sweep_stream(n_quads, seed=16990, t=3, replica=5, colour=1):
    out = np.empty(4 * n_quads, dtype=np.uint64)
    key = pyphilox.seed_key(seed)
    for q in range(n_quads):
        out[4 * q:4 * q + 4] = oracle.philox4x32_10((q, t, replica, colour), key)
    return out


@pytest.fixture(scope="module")
def stream():
    return _sweep_stream(1 << 16)  # 262144 uniforms


def test_uniform_histogram_100_bins(stream):
    # Supplementary S.5: 100-bin histogram of uniforms on [0, 1)
    u = stream.astype(np.float64) / 2**32
    counts, _ = np.histogram(u, bins=100, range=(0.0, 1.0))
    chi2, p = stats.chisquare(counts)
    assert p > 1e-3, (chi2, p)


def test_lag1_joint_histogram(stream):
    # Supplementary S.5: joint histogram of consecutive values
    u = stream.astype(np.float64) / 2**32
    h, _, _ = np.histogram2d(u[:-1:2], u[1::2], bins=10, range=[[0, 1], [0, 1]])
    chi2, p = stats.chisquare(h.ravel())
    assert p > 1e-3, (chi2, p)


def _bits(stream, n_words):
    w = stream[:n_words].astype(np.uint32)
    return np.unpackbits(w.view(np.uint8)).astype(np.int8)


def test_nist_frequency_monobit(stream):
    # NIST SP 800-22 section 2.1
    b = _bits(stream, 1 << 15)
    s = np.sum(2 * b.astype(np.int64) - 1)
    p = special.erfc(abs(s) / math.sqrt(len(b)) / math.sqrt(2))
    assert p > 1e-3


def test_nist_block_frequency(stream):
    # NIST SP 800-22 section 2.2, block length 128
    b = _bits(stream, 1 << 15)
    M = 128
    N = len(b) // M
    pi = b[: N * M].reshape(N, M).mean(axis=1)
    chi2 = 4 * M * np.sum((pi - 0.5) ** 2)
    p = special.gammaincc(N / 2, chi2 / 2)
    assert p > 1e-3


def test_nist_runs(stream):
    # NIST SP 800-22 section 2.3
    b = _bits(stream, 1 << 15).astype(np.int64)
    n = len(b)
    pi = b.mean()
    assert abs(pi - 0.5) < 2 / math.sqrt(n)
    v = 1 + np.count_nonzero(b[1:] != b[:-1])
    p = special.erfc(abs(v - 2 * n * pi * (1 - pi)) / (2 * math.sqrt(2 * n) * pi * (1 - pi)))
    assert p > 1e-3


def test_distinct_streams_are_uncorrelated():
    # Different colours / sweeps / replicas must not give the same words.
    a = _sweep_stream(2048, colour=0)
    b = _sweep_stream(2048, colour=1)
    c = _sweep_stream(2048, t=4)
    assert np.count_nonzero(a == b) < 5 and np.count_nonzero(b == c) < 5
    r = np.corrcoef(a.astype(np.float64), b.astype(np.float64))[0, 1]
    assert abs(r) < 4 / math.sqrt(len(a))
