"""Bit-exact parity at the full sizes of the three large workloads, in the
launch configuration the benchmark times (the autotuner's schedule, 100-sweep
calls, (B, M) every 100 sweeps), on this sampling plan:

- 256 x 1024^2: replicas 0, 36, 73, 109, 146, 182, 219 and 255 (the
  temperature range end to end) for the full 10^4 sweeps;
- uneven 512 (128^2 .. 8192^2): every replica for 5 sweeps under three
  schedules (the default mixed resident/streamed placement with graph replays
  of 2-sweep chunks; all replicas streamed, 32- and 64-bit words), and one
  replica of every size for the full 2000 sweeps;
- paper scale: every 512 x 528 replica for 20 sweeps, eight of them for the
  full 1000, and the 16384 x 12288 lattice for 50 sweeps.

The GPU runs each workload once per module; the oracle (large lattices split
over their rows on all host threads, which gives the same result for any
thread count) replays the sampled replicas.  Long oracle replays are cut into
chained 500-sweep pieces, one test each, each continuing from the oracle's own
state of the piece before.
"""
import os
import time

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

CHUNK = 500          # sweeps per chained oracle piece
CFG2_IDX = [0, 36, 73, 109, 146, 182, 219, 255]


def _note(msg):
    path = os.environ.get("ISING_PROGRESS_LOG")
    if path:
        with open(path, "a") as f:
            f.write(f"{time.strftime('%H:%M:%S')}   {msg}\n")
            f.flush()


def _odesc(r):
    return oracle.desc(r.Lx, r.Ly, r.J, r.beta, r.seed, r.replica, r.init, rng=r.rng)


def _batch(reps, schedule=None, autotune=False):
    import paper_2404_16990_amd as P
    b = P.Batch([dict(Lx=r.Lx, Ly=r.Ly, J=r.J, beta=r.beta, seed=r.seed, replica=r.replica, init=r.init, rng=r.rng)
                 for r in reps])
    if schedule:
        b.set_schedule(**schedule)
    if autotune:
        b.autotune(trial_sweeps=100)
    return b


def _run_calls(b, n, per_call, every, keep):
    """n sweeps as calls of per_call sweeps recording every `every`; returns
    the traces of rows `keep` (numpy, concatenated over calls)."""
    import torch
    bs, ms = [], []
    idx = torch.tensor(keep, device="cuda")
    for _ in range(n // per_call):
        gb, gm = b.run(per_call, every)
        bs.append(gb.index_select(0, idx).cpu().numpy())
        ms.append(gm.index_select(0, idx).cpu().numpy())
    torch.cuda.synchronize()
    return np.concatenate(bs, axis=1), np.concatenate(ms, axis=1)


# ---- a chained oracle replay shared by the pieces of one replica --------------------------

_oracle_states = {}


def _oracle_piece(key, desc, t0, n, every):
    """Sweeps t0 .. t0+n of the replica `key` on the oracle, continuing from the
    state the previous piece left (t0 = 0 starts from the initial state)."""
    if t0 == 0:
        _oracle_states[key] = (0, oracle.init_state(desc))
    t, s = _oracle_states[key]
    assert t == t0, f"piece {t0} of {key} needs the piece before it (state at {t})"
    b, m = oracle.sweeps_rows(desc, s, n, t0=t0, record_every=every)
    _oracle_states[key] = (t0 + n, s)
    return s, b, m


# ---- 256 x 1024^2, eight replicas for the full 10^4 sweeps ----------------------------------

@pytest.fixture(scope="module")
def cfg2():
    w = workloads.batch_256x1024()
    b = _batch(w.replicas, autotune=True)
    out = {"w": w, "sched": b.schedule, "bond": [], "mag": [], "spins": {}}
    for c in range(w.sweeps // CHUNK):
        gb, gm = _run_calls(b, CHUNK, 100, w.record_every, CFG2_IDX)
        out["bond"].append(gb)
        out["mag"].append(gm)
        out["spins"][c] = [b.get_spins(i) for i in CFG2_IDX]
    b.close()
    _note(f"256x1024^2: GPU run of 10^4 sweeps done under {out['sched']}")
    return out


@pytest.mark.parametrize("c", range(10000 // CHUNK))
@pytest.mark.parametrize("k", range(len(CFG2_IDX)))
def test_batch_256x1024_full_length(cfg2, k, c):
    w = cfg2["w"]
    i = CFG2_IDX[k]
    s, ob, om = _oracle_piece(("cfg2", i), _odesc(w.replicas[i]), c * CHUNK, CHUNK, w.record_every)
    assert np.array_equal(cfg2["bond"][c][k], ob) and np.array_equal(cfg2["mag"][c][k], om), (i, c)
    assert np.array_equal(cfg2["spins"][c][k], s), (i, c)
    _note(f"256x1024^2 replica {i} sweeps {c * CHUNK}..{(c + 1) * CHUNK} bit-exact")


# ---- uneven 512: every replica for 5 sweeps under three schedules ---------------------------

def _init_states(descs):
    """Oracle initial states on all host threads (the library calls release the GIL)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(oracle.default_threads()) as pool:
        return list(pool.map(oracle.init_state, descs))


@pytest.fixture(scope="module")
def uneven5():
    w = workloads.uneven_512()
    descs = [_odesc(r) for r in w.replicas]
    states = _init_states(descs)
    ob, om = oracle.run_batch(descs, states, 5, record_every=1)
    _note("uneven 512: oracle 5 sweeps of every replica done")
    return w, states, ob, om


@pytest.mark.parametrize("sched", [
    dict(use_graph=1, sweeps_per_launch=2),
    dict(resident_max_bytes=0, word_bits=32, use_graph=1, sweeps_per_launch=2),
    dict(resident_max_bytes=0, word_bits=64, use_graph=1, sweeps_per_launch=2),
], ids=["mixed_graph2", "streamed32_graph2", "streamed64_graph2"])
def test_uneven_512_all_replicas_5_sweeps(uneven5, sched):
    """Two replays of a captured 2-sweep chunk and a 1-sweep remainder."""
    import torch
    w, states, ob, om = uneven5
    b = _batch(w.replicas, sched)
    n_res, n_str = b.mode_counts()
    if "resident_max_bytes" in sched:
        assert n_res == 0
    else:
        assert n_res > 0 and n_str > 0
    gb, gm = b.run(5, 1)
    torch.cuda.synchronize()
    assert np.array_equal(gb.cpu().numpy(), ob) and np.array_equal(gm.cpu().numpy(), om)
    for i, s in enumerate(states):
        assert np.array_equal(b.get_spins(i), s), (i, w.replicas[i].Lx)
    assert b.graph_stats()[1] >= 1
    b.close()


# ---- uneven 512: one replica of every size for the full 2000 sweeps -------------------------

def _one_per_size(reps):
    seen = {}
    for i, r in enumerate(reps):
        seen.setdefault(r.Lx, i)
    return [seen[L] for L in sorted(seen)]


UNEVEN_SIZES = [128 << k for k in range(7)]


@pytest.fixture(scope="module")
def uneven_full():
    w = workloads.uneven_512()
    idx = _one_per_size(w.replicas)
    assert [w.replicas[i].Lx for i in idx] == UNEVEN_SIZES
    b = _batch(w.replicas, dict(resident_max_bytes=0), autotune=True)   # the benchmark's tuning start
    out = {"w": w, "idx": idx, "sched": b.schedule, "bond": [], "mag": [], "spins": {}}
    for c in range(w.sweeps // CHUNK):
        gb, gm = _run_calls(b, CHUNK, 100, w.record_every, idx)
        out["bond"].append(gb)
        out["mag"].append(gm)
        out["spins"][c] = [b.get_spins(i) for i in idx]
    b.close()
    _note(f"uneven 512: GPU run of 2000 sweeps done under {out['sched']}")
    return out


@pytest.mark.parametrize("c", range(2000 // CHUNK))
@pytest.mark.parametrize("L", UNEVEN_SIZES)
def test_uneven_512_one_per_size_full_length(uneven_full, L, c):
    w, idx = uneven_full["w"], uneven_full["idx"]
    k = UNEVEN_SIZES.index(L)
    i = idx[k]
    s, ob, om = _oracle_piece(("uneven", i), _odesc(w.replicas[i]), c * CHUNK, CHUNK, w.record_every)
    assert np.array_equal(uneven_full["bond"][c][k], ob) and np.array_equal(uneven_full["mag"][c][k], om), (i, c)
    assert np.array_equal(uneven_full["spins"][c][k], s), (i, L, c)
    _note(f"uneven 512 replica {i} ({L}^2) sweeps {c * CHUNK}..{(c + 1) * CHUNK} bit-exact")


# ---- paper scale: all small replicas x 20, eight x 1000, the big lattice x 50 ----------------

PAPER_FULL = [0, 107, 215, 322, 430, 537, 645, 753]


@pytest.fixture(scope="module")
def paper():
    w = workloads.paper_scale()
    big = len(w.replicas) - 1
    b = _batch(w.replicas, autotune=True)
    everyone = list(range(len(w.replicas)))
    out = {"w": w, "big": big, "sched": b.schedule}
    out["b20"], out["m20"] = _run_calls(b, 20, 20, 10, everyone)
    out["small20"] = [b.get_spins(i) for i in range(big)]
    out["b50"], out["m50"] = _run_calls(b, 30, 30, 10, everyone)
    out["big50"] = b.get_spins(big)
    out["b1000"], out["m1000"] = _run_calls(b, 950, 50, 50, PAPER_FULL)
    out["full"] = [b.get_spins(i) for i in PAPER_FULL]
    b.close()
    _note(f"paper scale: GPU run of 1000 sweeps done under {out['sched']}")
    return out


def test_paper_scale_all_small_replicas_20_sweeps(paper):
    w, big = paper["w"], paper["big"]
    descs = [_odesc(r) for r in w.replicas[:big]]
    states = _init_states(descs)
    ob, om = oracle.run_batch(descs, states, 20, record_every=10)
    assert np.array_equal(paper["b20"][:big], ob) and np.array_equal(paper["m20"][:big], om)
    for i, s in enumerate(states):
        assert np.array_equal(paper["small20"][i], s), i
    for i in PAPER_FULL:
        _oracle_states[("paper", i)] = (20, states[i])


def test_paper_scale_big_lattice_50_sweeps(paper):
    w, big = paper["w"], paper["big"]
    d = _odesc(w.replicas[big])
    s = oracle.init_state(d)
    ob, om = oracle.sweeps_rows(d, s, 20, record_every=10)
    assert np.array_equal(paper["b20"][big], ob) and np.array_equal(paper["m20"][big], om)
    ob, om = oracle.sweeps_rows(d, s, 30, t0=20, record_every=10)
    assert np.array_equal(paper["b50"][big], ob) and np.array_equal(paper["m50"][big], om)
    assert np.array_equal(paper["big50"], s)


def test_paper_scale_eight_small_replicas_full_length(paper):
    """Continues the oracle states of the 20-sweep test to sweep 1000."""
    w = paper["w"]
    for k, i in enumerate(PAPER_FULL):
        t, s = _oracle_states[("paper", i)]
        assert t == 20
        d = _odesc(w.replicas[i])
        ob, om = oracle.sweeps(d, s, 30, t0=20, record_every=10)
        assert np.array_equal(paper["b50"][i], ob) and np.array_equal(paper["m50"][i], om), i
        ob, om = oracle.sweeps(d, s, 950, t0=50, record_every=50)
        assert np.array_equal(paper["b1000"][k], ob) and np.array_equal(paper["m1000"][k], om), i
        assert np.array_equal(paper["full"][k], s), i
