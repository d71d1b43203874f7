"""The seeded synthetic workloads match the recipes stated for them: shapes,
counts, temperature grids, seeds, replica ids and start modes (CPU only)."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import workloads as W  # noqa: E402


def _valid_2d(reps):
    for r in reps:
        assert r.Lx % 64 == 0 and r.Ly % 2 == 0 and r.Ly >= 2 and r.J == 1.0 and r.T > 0


def test_single_64():
    w = W.single_64()
    assert [(r.Lx, r.Ly, r.T) for r in w.replicas] == [(64, 64, 2.269185)]
    assert (w.sweeps, w.record_every) == (1000, 1)


def test_batch_256x1024():
    w = W.batch_256x1024()
    _valid_2d(w.replicas)
    assert len(w.replicas) == 256 and w.spins == 256 * 1024 * 1024
    assert [r.replica for r in w.replicas] == list(range(256))
    assert len({r.seed for r in w.replicas}) == 256
    T = np.array([r.T for r in w.replicas])
    assert T[0] == 1.5 and T[-1] == pytest.approx(3.5) and np.all(np.diff(T) > 0)
    assert all(r.init == W.INIT_RANDOM for r in w.replicas)


def test_uneven_512():
    w = W.uneven_512()
    _valid_2d(w.replicas)
    assert len(w.replicas) == 512
    sides = {r.Lx for r in w.replicas}
    assert sides == {1 << k for k in range(7, 14)}  # every size 128 .. 8192 drawn
    assert all(r.Lx == r.Ly for r in w.replicas)
    assert w.spins == 6_899_056_640
    T = np.array([r.T for r in w.replicas])
    assert T.min() >= 2.0 and T.max() < 2.6
    assert W.uneven_512().spins == w.spins  # seeded: the same draw every time


def test_paper_scale():
    w = W.paper_scale()
    _valid_2d(w.replicas)
    small, big = w.replicas[:-1], w.replicas[-1]
    assert len(small) == 754 and all((r.Lx, r.Ly) == (512, 528) for r in small)
    assert (big.Lx, big.Ly, big.T, big.replica) == (16384, 12288, 2.269185, 754)
    T = np.array([r.T for r in small])
    assert T[0] == 1.8 and T[-1] == pytest.approx(3.0) and np.allclose(np.diff(T), 1.2 / 753)
    assert all(r.init == W.INIT_UP for r in w.replicas)
    assert w.spins == 405_159_936


def test_learned_64x256():
    w = W.learned_64x256()
    _valid_2d(w.replicas)
    assert len(w.replicas) == 64 and all((r.Lx, r.Ly) == (256, 256) for r in w.replicas)
    assert len(W.LEARNED_TEMPS) == 8 and W.T_CRITICAL_PRINTED in W.LEARNED_TEMPS
    assert min(W.LEARNED_TEMPS) == 2.20 and max(W.LEARNED_TEMPS) == 2.35
    for g, T in enumerate(W.LEARNED_TEMPS):
        group = w.replicas[8 * g: 8 * g + 8]
        assert all(r.T == T for r in group)
    assert len({r.seed for r in w.replicas}) == 64  # independent chains


def test_cubic_16x256():
    w = W.cubic_16x256()
    assert len(w.replicas) == 16 and all((r.Lx, r.Ly, r.Lz) == (256, 256, 256) for r in w.replicas)
    T = np.array([r.T for r in w.replicas])
    assert T[0] == 3.5 and T[-1] == pytest.approx(5.5)
    assert T.min() < 4.51 < T.max()  # brackets the 3D critical temperature


def test_seeded_helpers():
    a, b = W.random_pm1((5, 7), 3), W.random_pm1((5, 7), 3)
    assert np.array_equal(a, b) and set(np.unique(a)) <= {-1, 1}
    for Lx, Ly in W.small_shapes(1, 50):
        assert Lx % 64 == 0 and Ly % 2 == 0 and 2 <= Ly <= 40 and 64 <= Lx <= 256
    p = W.nn_initial_params(64)
    assert p.dtype == np.float32 and p.size == 62_337  # the network's parameter count
    assert np.array_equal(p, W.nn_initial_params(64))
