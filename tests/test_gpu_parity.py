"""Bit-exact parity of the HIP library (through its C ABI) with the CPU oracle.

Every case compares lattice states and (B, M) traces element by element on the
same seeded inputs; the GPU side runs under several execution schedules, all of
which must give identical results (word width, LDS-resident vs streaming,
workgroup shape, graph replay vs direct launches, sweeps per launch).
"""
import math

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

SCHEDULES = {
    "default": {},
    "stream32": dict(resident_max_bytes=0, word_bits=32),
    "stream64": dict(resident_max_bytes=0, word_bits=64),
    "resident64": dict(word_bits=64),
    "eager": dict(use_graph=0, sweeps_per_launch=4),
    "stream_small_wg": dict(resident_max_bytes=0, stream_threads=64, stream_words=64, sweeps_per_launch=3),
    "stream_big_wg": dict(resident_max_bytes=0, stream_threads=1024, stream_words=4096, word_bits=64),
    "resident1024": dict(resident_threads=1024, sweeps_per_launch=7),
    "resident64t": dict(resident_threads=64, sweeps_per_launch=1),
}


def _P():
    import paper_2404_16990_amd as P
    return P


def gdesc(r):
    return dict(Lx=r.Lx, Ly=r.Ly, J=r.J, beta=r.beta, seed=r.seed, replica=r.replica, init=r.init, rng=r.rng)


def odesc(r):
    return oracle.desc(r.Lx, r.Ly, r.J, r.beta, r.seed, r.replica, r.init, rng=r.rng)


def gpu_batch(reps, schedule=None):
    P = _P()
    b = P.Batch([gdesc(r) for r in reps])
    if schedule:
        b.set_schedule(**schedule)
    return b


def gpu_run(b, n, record_every=0):
    import torch
    out = b.run(n, record_every)
    torch.cuda.synchronize()
    if out is None:
        return None, None
    return out[0].cpu().numpy(), out[1].cpu().numpy()


def oracle_run(reps, n, record_every=0, states=None, t0=None):
    descs = [odesc(r) for r in reps]
    if states is None:
        states = [oracle.init_state(d) for d in descs]
    b, m = oracle.run_batch(descs, states, n, t0=t0, record_every=record_every)
    return states, b, m


def assert_states(b, reps, states, which=None):
    for i in (which if which is not None else range(len(reps))):
        g = b.get_spins(i)
        assert np.array_equal(g, states[i]), f"state mismatch in replica {i} ({reps[i].Lx}x{reps[i].Ly})"


# ---- config: one 64x64 lattice at T_c, 1000 sweeps, every sweep recorded ---------

@pytest.mark.parametrize("sched", list(SCHEDULES))
def test_single_64_full_trace(sched):
    w = workloads.single_64()
    b = gpu_batch(w.replicas, SCHEDULES[sched])
    gb, gm = gpu_run(b, w.sweeps, w.record_every)
    states, ob, om = oracle_run(w.replicas, w.sweeps, w.record_every)
    assert np.array_equal(gb, ob) and np.array_equal(gm, om)
    assert_states(b, w.replicas, states)
    assert b.get_sweep(0) == w.sweeps


# ---- initial states ----------------------------------------------------------------

def test_initial_states_match_oracle():
    reps = [workloads.Replica(64 * (1 + i % 3), 2 + 2 * i, 2.0 + 0.1 * i, 1000 + i, i,
                              [workloads.INIT_RANDOM, workloads.INIT_UP, workloads.INIT_DOWN][i % 3])
            for i in range(9)]
    b = gpu_batch(reps)
    for i, r in enumerate(reps):
        assert np.array_equal(b.get_spins(i), oracle.init_state(odesc(r))), i
    gb, gm = b.observables()
    for i, r in enumerate(reps):
        assert (gb[i], gm[i]) == oracle.observables(oracle.init_state(odesc(r)))


# ---- random small shapes, mixed temperatures and starts ----------------------------

def _random_reps(seed, count):
    rng = np.random.default_rng(seed)
    shapes = workloads.small_shapes(seed, count)
    reps = []
    for i, (Lx, Ly) in enumerate(shapes):
        reps.append(workloads.Replica(Lx, Ly, float(rng.uniform(1.0, 4.0)), int(rng.integers(0, 2**63)),
                                      int(rng.integers(0, 2**32)), int(rng.integers(0, 3)),
                                      J=float(rng.choice([1.0, 0.5, 1.7]))))
    return reps


@pytest.mark.parametrize("sched", list(SCHEDULES))
def test_random_shapes(sched):
    reps = _random_reps(101, 14)
    b = gpu_batch(reps, SCHEDULES[sched])
    gb, gm = gpu_run(b, 25, 5)
    states, ob, om = oracle_run(reps, 25, 5)
    assert np.array_equal(gb, ob) and np.array_equal(gm, om)
    assert_states(b, reps, states)


def test_edge_shapes_and_ragged_tiles():
    # smallest lattices, odd word counts (64-bit falls back to 32 there), tall strips
    reps = [workloads.Replica(64, 2, 2.2, 1, 0), workloads.Replica(192, 2, 1.1, 2, 1),
            workloads.Replica(64, 130, 3.3, 3, 2), workloads.Replica(320, 18, 2.5, 4, 3),
            workloads.Replica(1088, 6, 2.0, 5, 4, workloads.INIT_UP)]
    for sched in ("default", "stream64", "stream_small_wg", "resident64t"):
        b = gpu_batch(reps, SCHEDULES[sched])
        gb, gm = gpu_run(b, 11, 1)
        states, ob, om = oracle_run(reps, 11, 1)
        assert np.array_equal(gb, ob) and np.array_equal(gm, om), sched
        assert_states(b, reps, states)


# ---- run composition, record cadence, checkpoint/resume ------------------------------

def test_split_runs_equal_one_run():
    reps = _random_reps(7, 6)
    b = gpu_batch(reps, dict(sweeps_per_launch=4))
    gpu_run(b, 7, 1)
    gb, gm = gpu_run(b, 13, 13)
    gpu_run(b, 0)
    states, ob, om = oracle_run(reps, 20, 1)
    assert np.array_equal(gb[:, 0], ob[:, 19]) and np.array_equal(gm[:, 0], om[:, 19])
    assert_states(b, reps, states)
    assert all(b.get_sweep(i) == 20 for i in range(len(reps)))


def test_record_every_not_dividing_run():
    reps = _random_reps(8, 4)
    b = gpu_batch(reps)
    gb, gm = gpu_run(b, 23, 5)  # records after sweeps 5, 10, 15, 20
    states, ob, om = oracle_run(reps, 23, 5)
    assert gb.shape == (4, 4) and np.array_equal(gb, ob) and np.array_equal(gm, om)
    assert_states(b, reps, states)


def test_observables_after_run():
    reps = _random_reps(9, 8)
    b = gpu_batch(reps, SCHEDULES["stream64"])
    gpu_run(b, 9)
    states, _, _ = oracle_run(reps, 9)
    gb, gm = b.observables()
    for i, s in enumerate(states):
        assert (gb[i], gm[i]) == oracle.observables(s)


def test_checkpoint_resume():
    reps = _random_reps(11, 5)
    a = gpu_batch(reps)
    gpu_run(a, 10)
    saved = [(a.get_spins(i), a.get_sweep(i)) for i in range(len(reps))]
    b = gpu_batch(reps, SCHEDULES["stream32"])
    for i, (s, t) in enumerate(saved):
        b.set_spins(i, s)
        b.set_sweep(i, t)
    gb, gm = gpu_run(b, 15, 3)
    states, ob, om = oracle_run(reps, 25, 1)
    assert np.array_equal(gb, ob[:, 12::3]) and np.array_equal(gm, om[:, 12::3])
    assert_states(b, reps, states)


def test_set_spins_then_run_from_arbitrary_state():
    reps = [workloads.Replica(128, 12, 2.4, 5, 1)]
    b = gpu_batch(reps)
    s0 = workloads.random_pm1((12, 128), seed=77)
    b.set_spins(0, s0)
    gb, gm = gpu_run(b, 6, 1)
    s = s0.copy()
    ob, om = oracle.sweeps(odesc(reps[0]), s, 6, record_every=1)
    assert np.array_equal(gb[0], ob) and np.array_equal(gm[0], om)
    assert np.array_equal(b.get_spins(0), s)


def test_set_spins_rejects_bad_values():
    P = _P()
    b = gpu_batch([workloads.Replica(64, 4, 2.0, 1, 0)])
    before = b.get_spins(0)
    bad = before.copy()
    bad[1, 3] = 0
    with pytest.raises(P.IsingError) as e:
        b.set_spins(0, bad)
    assert e.value.code == P.ISING_E_INVALID
    assert np.array_equal(b.get_spins(0), before)


def test_sweep_counter_limit():
    P = _P()
    b = gpu_batch([workloads.Replica(64, 4, 2.0, 1, 0)])
    b.set_sweep(0, 2**32 - 3)
    with pytest.raises(P.IsingError):
        b.run(5)
    gpu_run(b, 2)  # reaches 2^32 - 1
    s = oracle.init_state(odesc(workloads.Replica(64, 4, 2.0, 1, 0)))
    oracle.sweeps(odesc(workloads.Replica(64, 4, 2.0, 1, 0)), s, 2, t0=2**32 - 3)
    assert np.array_equal(b.get_spins(0), s)


# ---- special temperatures and couplings ---------------------------------------------

def test_special_temperatures():
    reps = [workloads.Replica(128, 8, 1.0, 3, 0), workloads.Replica(64, 6, 1.0, 4, 1),
            workloads.Replica(64, 10, 2.0, 5, 2, workloads.INIT_UP, J=0.25)]
    descs = [gdesc(r) for r in reps]
    descs[0]["beta"] = 0.0          # T = infinity: every proposal accepted
    descs[1]["beta"] = math.inf     # T = 0
    P = _P()
    b = P.Batch(descs)
    gb, gm = gpu_run(b, 5, 1)
    od = [oracle.desc(d["Lx"], d["Ly"], d["J"], d["beta"], d["seed"], d["replica"], d["init"]) for d in descs]
    states = [oracle.init_state(d) for d in od]
    ob, om = oracle.run_batch(od, states, 5, record_every=1)
    assert np.array_equal(gb, ob) and np.array_equal(gm, om)
    for i in range(3):
        assert np.array_equal(b.get_spins(i), states[i])


def test_set_beta_mid_run():
    reps = _random_reps(12, 3)
    b = gpu_batch(reps)
    gpu_run(b, 4)
    b.set_beta(1, 0.9)
    gpu_run(b, 5)
    descs = [odesc(r) for r in reps]
    states = [oracle.init_state(d) for d in descs]
    oracle.run_batch(descs, states, 4)
    descs[1] = oracle.desc(reps[1].Lx, reps[1].Ly, reps[1].J, 0.9, reps[1].seed, reps[1].replica, reps[1].init)
    oracle.run_batch(descs, states, 5, t0=4)
    assert_states(b, reps, states)


# ---- full-size workload in the benchmark's launch configuration ----------------------

def test_batch_256x1024_all_replicas_20_sweeps():
    w = workloads.batch_256x1024()
    b = gpu_batch(w.replicas)
    gb, gm = gpu_run(b, 20, 10)
    states, ob, om = oracle_run(w.replicas, 20, 10)
    assert np.array_equal(gb, ob) and np.array_equal(gm, om)
    assert_states(b, w.replicas, states, which=range(0, 256, 17))


# ---- autotuner: state untouched, self-checked candidates, cache ---------------------

def test_autotune_leaves_state_and_keeps_parity(tmp_path, monkeypatch):
    monkeypatch.setenv("ISING_AUTOTUNE_CACHE", str(tmp_path / "tune.txt"))
    reps = _random_reps(21, 6) + [workloads.Replica(1024, 64, 2.3, 9, 99)]
    b = gpu_batch(reps)
    gpu_run(b, 3)
    before = [b.get_spins(i) for i in range(len(reps))]
    sched, n_tried = b.autotune(trial_sweeps=4)
    assert n_tried >= 6
    assert [b.get_sweep(i) for i in range(len(reps))] == [3] * len(reps)
    for i, s in enumerate(before):
        assert np.array_equal(b.get_spins(i), s)
    assert b.schedule == sched
    gb, gm = gpu_run(b, 9, 3)
    states, ob, om = oracle_run(reps, 12, 1)
    assert np.array_equal(gb, ob[:, 5::3]) and np.array_equal(gm, om[:, 5::3])
    assert_states(b, reps, states)
    # same shapes again: served from the cache file without timing
    b2 = gpu_batch(reps)
    sched2, n2 = b2.autotune(trial_sweeps=4)
    assert n2 == 0 and sched2 == sched


# (the uneven 512-replica and paper-scale batches at full size: test_gpu_parity_scale.py)


# ---- hipGraph replays interleaved with eager work --------------------------------------

def test_graph_replays_between_eager_calls():
    """Every replay of a captured chunk is checked against the oracle, with eager
    library work (observables, spin reads, a beta change) and host synchronisation
    between replays."""
    reps = _random_reps(31, 5)
    b = gpu_batch(reps, dict(use_graph=1, sweeps_per_launch=3))
    descs = [odesc(r) for r in reps]
    states = [oracle.init_state(d) for d in descs]
    t = 0
    for k in range(6):
        gb, gm = gpu_run(b, 9, 3)  # three replays of the same 3-sweep graph
        ob, om = oracle.run_batch(descs, states, 9, t0=t, record_every=3)
        t += 9
        assert np.array_equal(gb, ob) and np.array_equal(gm, om), k
        B, M = b.observables()
        for i, s in enumerate(states):
            assert (B[i], M[i]) == oracle.observables(s)
        assert np.array_equal(b.get_spins(k % 5), states[k % 5])
        if k == 2:
            b.set_beta(1, 0.77)
            descs[1] = oracle.desc(reps[1].Lx, reps[1].Ly, reps[1].J, 0.77, reps[1].seed, reps[1].replica, reps[1].init)
    assert_states(b, reps, states)
