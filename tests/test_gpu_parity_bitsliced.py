"""Bit-exact parity with the oracle under the bit-sliced random-number
contract (rng = 1): each site's uniform is its bit of the 32 transposed words
of its 32-site group, and the GPU draws only the words needed to decide every
site of a wave (most significant bit first).  The same cases as the site
contract: full trace of the 64^2 configuration under every schedule, random
and edge shapes, special temperatures, mixed contracts in one batch, and the
benchmark batch in its launch configuration.
"""
import dataclasses
import math

import numpy as np
import pytest

import oracle
import workloads
from test_gpu_parity import (SCHEDULES, _P, _random_reps, assert_states, gdesc, gpu_batch, gpu_run, odesc,
                             oracle_run)

pytestmark = pytest.mark.gpu


def _bs(reps):
    return [dataclasses.replace(r, rng=1) for r in reps]


@pytest.mark.parametrize("sched", list(SCHEDULES))
def test_single_64_full_trace_bitsliced(sched):
    w = workloads.single_64()
    reps = _bs(w.replicas)
    b = gpu_batch(reps, SCHEDULES[sched])
    gb, gm = gpu_run(b, w.sweeps, w.record_every)
    states, ob, om = oracle_run(reps, w.sweeps, w.record_every)
    assert np.array_equal(gb, ob) and np.array_equal(gm, om)
    assert_states(b, reps, states)


@pytest.mark.parametrize("sched", ["default", "stream32", "stream64", "resident64t", "eager"])
def test_random_shapes_bitsliced(sched):
    reps = _bs(_random_reps(202, 14))
    b = gpu_batch(reps, SCHEDULES[sched])
    gb, gm = gpu_run(b, 25, 5)
    states, ob, om = oracle_run(reps, 25, 5)
    assert np.array_equal(gb, ob) and np.array_equal(gm, om)
    assert_states(b, reps, states)


def test_mixed_contracts_in_one_batch():
    reps = _random_reps(303, 8)
    reps = [dataclasses.replace(r, rng=i % 2) for i, r in enumerate(reps)]
    for sched in ("default", "stream64"):
        b = gpu_batch(reps, SCHEDULES[sched])
        gb, gm = gpu_run(b, 12, 3)
        states, ob, om = oracle_run(reps, 12, 3)
        assert np.array_equal(gb, ob) and np.array_equal(gm, om), sched
        assert_states(b, reps, states)


def test_edge_shapes_and_special_temperatures_bitsliced():
    reps = _bs([workloads.Replica(64, 2, 2.2, 1, 0), workloads.Replica(192, 2, 1.1, 2, 1),
                workloads.Replica(64, 130, 3.3, 3, 2), workloads.Replica(1088, 6, 0.6, 5, 4, workloads.INIT_UP)])
    descs = [gdesc(r) for r in reps] + [dict(gdesc(reps[0]), beta=0.0, replica=9),
                                        dict(gdesc(reps[1]), beta=math.inf, replica=10)]
    P = _P()
    b = P.Batch(descs)
    gb, gm = gpu_run(b, 9, 1)
    od = [oracle.desc(d["Lx"], d["Ly"], d["J"], d["beta"], d["seed"], d["replica"], d["init"], rng=1)
          for d in descs]
    states = [oracle.init_state(d) for d in od]
    ob, om = oracle.run_batch(od, states, 9, record_every=1)
    assert np.array_equal(gb, ob) and np.array_equal(gm, om)
    for i in range(len(descs)):
        assert np.array_equal(b.get_spins(i), states[i]), i


def test_batch_256x1024_bitsliced_20_sweeps():
    w = workloads.batch_256x1024()
    reps = _bs(w.replicas)
    b = gpu_batch(reps)
    gb, gm = gpu_run(b, 20, 10)
    idx = list(range(0, 256, 15))
    states, ob, om = oracle_run([reps[i] for i in idx], 20, 10)
    assert np.array_equal(gb[idx], ob) and np.array_equal(gm[idx], om)
    for k, i in enumerate(idx):
        assert np.array_equal(b.get_spins(i), states[k]), i


def test_rng_field_is_validated():
    P = _P()
    d = gdesc(workloads.Replica(64, 4, 2.0, 1, 0))
    d["rng"] = 2
    with pytest.raises(P.IsingError):
        P.Batch([d])
