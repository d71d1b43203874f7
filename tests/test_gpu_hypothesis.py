"""Property-based parity: hypothesis draws small batches (shapes, temperatures
including beta = 0 and infinity, seeds, starts, random-number contracts,
execution schedules, run lengths and recording cadences) and every draw must
be bit-exact with the CPU oracle, through the C ABI, for the 2D sweeps, the
cluster steps and the 3D sweeps.  Draws are derandomized (the same cases on
every run) and no example database is written.
"""
import math

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle

pytestmark = pytest.mark.gpu

SETTINGS = settings(max_examples=100, deadline=None, derandomize=True, database=None,
                    suppress_health_check=list(HealthCheck))

SCHEDULES = [
    {},
    dict(resident_max_bytes=0, word_bits=32),
    dict(resident_max_bytes=0, word_bits=64, stream_threads=64, stream_words=64, sweeps_per_launch=3),
    dict(word_bits=64, resident_threads=64, sweeps_per_launch=1),
    dict(use_graph=0, sweeps_per_launch=4),
]

betas = st.one_of(st.sampled_from([0.0, math.inf]), st.floats(0.05, 1.5))


def _P():
    import paper_2404_16990_amd as P
    return P


def _sync_np(out):
    import torch
    torch.cuda.synchronize()
    return (out[0].cpu().numpy(), out[1].cpu().numpy()) if out is not None else (None, None)


replica2d = st.tuples(st.integers(1, 6), st.integers(1, 40), betas, st.integers(0, 2 ** 64 - 1),
                      st.integers(0, 2), st.integers(0, 1))


@SETTINGS
@given(reps=st.lists(replica2d, min_size=1, max_size=3), sched=st.integers(0, len(SCHEDULES) - 1),
       n=st.integers(1, 8), every=st.integers(0, 3))
def test_sweeps_2d(reps, sched, n, every):
    print(f"2d reps={reps} sched={sched} n={n} every={every}", flush=True)
    g = [dict(Lx=64 * w, Ly=2 * h, J=1.0, beta=beta, seed=seed, replica=i, init=init, rng=rng)
         for i, (w, h, beta, seed, init, rng) in enumerate(reps)]
    o = [oracle.desc(64 * w, 2 * h, 1.0, beta, seed, i, init, rng=rng)
         for i, (w, h, beta, seed, init, rng) in enumerate(reps)]
    b = _P().Batch(g)
    try:
        if SCHEDULES[sched]:
            b.set_schedule(**SCHEDULES[sched])
        gb, gm = _sync_np(b.run(n, every))
        states = [oracle.init_state(d) for d in o]
        ob, om = oracle.run_batch(o, states, n, record_every=every)
        if every:
            np.testing.assert_array_equal(gb, ob)
            np.testing.assert_array_equal(gm, om)
        for i, s in enumerate(states):
            assert np.array_equal(b.get_spins(i), s), i
    finally:
        b.close()


replica_cl = st.tuples(st.integers(1, 4), st.integers(1, 75), betas, st.integers(0, 2 ** 64 - 1),
                       st.integers(0, 2))


@SETTINGS
@given(reps=st.lists(replica_cl, min_size=1, max_size=3), algo=st.sampled_from(["sw", "wolff"]),
       sweeps=st.integers(0, 3), n=st.integers(1, 4))
def test_cluster_steps(reps, algo, sweeps, n):
    print(f"cluster reps={reps} algo={algo} sweeps={sweeps} n={n}", flush=True)
    g = [dict(Lx=64 * w, Ly=2 * h, J=1.0, beta=beta, seed=seed, replica=i, init=init)
         for i, (w, h, beta, seed, init) in enumerate(reps)]
    o = [oracle.desc(64 * w, 2 * h, 1.0, beta, seed, i, init) for i, (w, h, beta, seed, init) in enumerate(reps)]
    b = _P().Batch(g)
    try:
        states = [oracle.init_state(d) for d in o]
        if sweeps:  # Metropolis sweeps first: the cluster steps continue the shared counter
            _sync_np(b.run(sweeps, 0))
            oracle.run_batch(o, states, sweeps)
        gb, gm = _sync_np(b.cluster(n, algo, 1))
        ob, om = oracle.run_cluster_batch(o, states, n, oracle.SWENDSEN_WANG if algo == "sw" else oracle.WOLFF,
                                          t0=sweeps, record_every=1)
        np.testing.assert_array_equal(gb, ob)
        np.testing.assert_array_equal(gm, om)
        for i, s in enumerate(states):
            assert np.array_equal(b.get_spins(i), s), i
    finally:
        b.close()


replica3d = st.tuples(st.sampled_from([1, 2, 3, 4, 8]), st.integers(1, 7), st.integers(1, 7), betas,
                      st.integers(0, 2 ** 64 - 1), st.integers(0, 2), st.integers(0, 1))


@SETTINGS
@given(reps=st.lists(replica3d, min_size=1, max_size=3), n=st.integers(1, 5), every=st.integers(1, 2))
def test_sweeps_3d(reps, n, every):
    print(f"3d reps={reps} n={n} every={every}", flush=True)
    g = [dict(Lx=64 * w, Ly=2 * h, Lz=2 * z, J=1.0, beta=beta, seed=seed, replica=i, init=init, rng=rng)
         for i, (w, h, z, beta, seed, init, rng) in enumerate(reps)]
    o = [oracle.desc3(64 * w, 2 * h, 2 * z, 1.0, beta, seed, i, init, rng=rng)
         for i, (w, h, z, beta, seed, init, rng) in enumerate(reps)]
    b = _P().Batch3(g)
    try:
        gb, gm = _sync_np(b.run(n, every))
        states = [oracle.init_state3(d) for d in o]
        ob, om = oracle.run_batch3(o, states, n, record_every=every)
        np.testing.assert_array_equal(gb, ob)
        np.testing.assert_array_equal(gm, om)
        for i, s in enumerate(states):
            assert np.array_equal(b.get_spins(i), s), i
    finally:
        b.close()
