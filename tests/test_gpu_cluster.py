"""Bit-exact parity of the cluster steps (Swendsen-Wang, Wolff) of the HIP
library, through its C ABI, with the CPU oracle.

Every case compares lattice states and (B, M) traces element by element on the
same seeded inputs: single lattices of every tile shape (one and several tiles
across and down, ragged last tile rows, Ly = 2 double bonds), the special
temperatures (beta = 0: no bonds; beta = infinity: every aligned bond),
batches mixing sizes, temperatures and algorithms with Metropolis sweeps
interleaved on the shared counter, the benchmark batch (256 x 1024^2) on
sampled replicas, and the largest accepted lattice under exact properties.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import philox

pytestmark = pytest.mark.gpu

ALGOS = {"sw": oracle.SWENDSEN_WANG, "wolff": oracle.WOLFF}


def _P():
    import paper_2404_16990_amd as P
    return P


def _descs(shapes):
    """shapes: list of (Lx, Ly, beta, seed, init)."""
    g = [dict(Lx=Lx, Ly=Ly, J=1.0, beta=beta, seed=seed, replica=i, init=init)
         for i, (Lx, Ly, beta, seed, init) in enumerate(shapes)]
    o = [oracle.desc(Lx, Ly, 1.0, beta, seed, i, init) for i, (Lx, Ly, beta, seed, init) in enumerate(shapes)]
    return g, o


def _gpu_cluster(b, n, algo, every):
    import torch
    out = b.cluster(n, algo, every)
    torch.cuda.synchronize()
    if out is None:
        return None, None
    return out[0].cpu().numpy(), out[1].cpu().numpy()


def _check_states(b, states, which=None):
    for i in (range(len(states)) if which is None else which):
        g = b.get_spins(i)
        assert np.array_equal(g, states[i]), f"state mismatch in replica {i} {states[i].shape}"


SHAPES = [(64, 2), (64, 4), (64, 32), (64, 34), (128, 64), (192, 96), (256, 256), (64, 130), (320, 62)]


@pytest.mark.parametrize("algo", list(ALGOS))
@pytest.mark.parametrize("beta", [0.25, 1.0 / 2.269185314213022, 0.6, 1.5])
def test_single_shapes(algo, beta):
    print(f"cluster {algo} beta={beta}", flush=True)
    g, o = _descs([(Lx, Ly, beta, 100 + i, 0) for i, (Lx, Ly) in enumerate(SHAPES)])
    P = _P()
    b = P.Batch(g)
    bond, mag = _gpu_cluster(b, 6, algo, 1)
    states = [oracle.init_state(d) for d in o]
    ob, om = oracle.run_cluster_batch(o, states, 6, ALGOS[algo], record_every=1)
    np.testing.assert_array_equal(bond, ob)
    np.testing.assert_array_equal(mag, om)
    _check_states(b, states)
    b.close()


@pytest.mark.parametrize("algo", list(ALGOS))
def test_special_temperatures(algo):
    """beta = 0 (every site its own cluster), beta = infinity from hot, cold
    and down starts (every aligned bond occupied)."""
    shapes = [(128, 66, 0.0, 7, 0), (64, 64, math.inf, 8, 0), (64, 64, math.inf, 9, 1),
              (192, 34, math.inf, 10, 2), (64, 2, math.inf, 11, 0), (64, 2, 0.0, 12, 0)]
    g, o = _descs(shapes)
    P = _P()
    b = P.Batch(g)
    bond, mag = _gpu_cluster(b, 5, algo, 1)
    states = [oracle.init_state(d) for d in o]
    ob, om = oracle.run_cluster_batch(o, states, 5, ALGOS[algo], record_every=1)
    np.testing.assert_array_equal(bond, ob)
    np.testing.assert_array_equal(mag, om)
    _check_states(b, states)
    b.close()


def test_mixed_batch_interleaved_with_sweeps():
    """A batch of 40 replicas of mixed shapes and temperatures: SW steps, then
    Metropolis sweeps (site and bit-sliced contracts), then Wolff steps, with
    one counter per replica shared by both kinds of update."""
    rng = np.random.default_rng(5)
    shapes = []
    for i in range(40):
        Lx = int(64 * rng.integers(1, 5))
        Ly = int(2 * rng.integers(1, 60))
        T = float(rng.uniform(1.2, 4.0))
        shapes.append((Lx, Ly, 1.0 / T, 1000 + i, int(rng.integers(0, 3))))
    g, o = _descs(shapes)
    for i in range(40):
        g[i]["rng"] = i % 2
        o[i].rng = i % 2
    P = _P()
    b = P.Batch(g)
    states = [oracle.init_state(d) for d in o]
    _, _ = _gpu_cluster(b, 4, "sw", 0)
    oracle.run_cluster_batch(o, states, 4, oracle.SWENDSEN_WANG)
    import torch
    b.run(3)
    torch.cuda.synchronize()
    oracle.run_batch(o, states, 3, t0=4)
    bond, mag = _gpu_cluster(b, 6, "wolff", 2)
    ob, om = oracle.run_cluster_batch(o, states, 6, oracle.WOLFF, t0=7, record_every=2)
    np.testing.assert_array_equal(bond, ob)
    np.testing.assert_array_equal(mag, om)
    _check_states(b, states)
    assert all(b.get_sweep(i) == 13 for i in range(40))
    b.close()


def test_split_calls_equal_one_call_and_workspace_reuse():
    g, o = _descs([(128, 96, 0.44, 3, 0), (64, 64, 0.5, 4, 0)])
    P = _P()
    b1, b2 = P.Batch(g), P.Batch(g)
    _gpu_cluster(b1, 5, "sw", 0)
    for _ in range(5):
        _gpu_cluster(b2, 1, "sw", 0)
    for i in range(2):
        assert np.array_equal(b1.get_spins(i), b2.get_spins(i))
    b1.close()
    b2.close()


def test_large_lattices_at_tc():
    """Four lattices of 2^20 sites at T_c (percolating clusters spanning many
    tiles): three Swendsen-Wang steps, then three Wolff steps."""
    Tc = 2.269185314213022
    shapes = [(1024, 1024, 1.0 / Tc, 50 + i, 0) for i in range(3)] + [(2048, 512, 1.0 / Tc, 60, 1)]
    g, o = _descs(shapes)
    P = _P()
    b = P.Batch(g)
    states = [oracle.init_state(d) for d in o]
    for t0, algo in [(0, "sw"), (3, "wolff")]:
        print(f"large {algo}", flush=True)
        bond, mag = _gpu_cluster(b, 3, algo, 1)
        ob, om = oracle.run_cluster_batch(o, states, 3, ALGOS[algo], t0=t0, record_every=1)
        np.testing.assert_array_equal(bond, ob)
        np.testing.assert_array_equal(mag, om)
        _check_states(b, states)
    b.close()


def test_batch_256x1024_sampled_replicas():
    """The benchmark batch (256 x 1024^2, T in [1.5, 3.5], random starts): 3 SW
    steps of the whole batch, 6 replicas across the temperature range compared
    in full with the oracle."""
    import workloads
    w = workloads.batch_256x1024()
    P = _P()
    g = [dict(Lx=r.Lx, Ly=r.Ly, J=r.J, beta=r.beta, seed=r.seed, replica=r.replica, init=r.init, rng=r.rng)
         for r in w.replicas]
    b = P.Batch(g)
    bond, mag = _gpu_cluster(b, 3, "sw", 1)
    pick = [0, 51, 102, 153, 204, 255]
    o = [oracle.desc(w.replicas[i].Lx, w.replicas[i].Ly, w.replicas[i].J, w.replicas[i].beta, w.replicas[i].seed,
                     w.replicas[i].replica, w.replicas[i].init, rng=w.replicas[i].rng) for i in pick]
    states = [oracle.init_state(d) for d in o]
    ob, om = oracle.run_cluster_batch(o, states, 3, oracle.SWENDSEN_WANG, record_every=1)
    np.testing.assert_array_equal(bond[pick], ob)
    np.testing.assert_array_equal(mag[pick], om)
    for k, i in enumerate(pick):
        assert np.array_equal(b.get_spins(i), states[k]), i
    b.close()


def test_argument_validation():
    import torch
    P = _P()
    b = P.Batch([dict(Lx=64, Ly=4, beta=0.4, seed=1, replica=0)])
    need = P.ising_cluster_ws_bytes(b.h)
    assert need >= 64 * 4 * 4 + 16
    ws = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    base = ws.data_ptr()
    aligned = (base + 255) & ~255
    for args, code in [((5, 1, 0, aligned, need), P.ISING_E_INVALID),
                       ((0, 1, 0, None, need), P.ISING_E_INVALID),
                       ((0, 1, 0, aligned + 64, need), P.ISING_E_INVALID),
                       ((0, 1, 0, aligned, need - 1), P.ISING_E_NOMEM),
                       ((0, 2 ** 32, 0, aligned, need), P.ISING_E_INVALID)]:
        with pytest.raises(P.IsingError) as e:
            P.ising_batch_cluster(b.h, *args, None, None, b._s())
        assert e.value.code == code
    assert b.get_sweep(0) == 0
    b.close()


def test_largest_lattice_exact_properties():
    """65536 x 65534 (Lx*Ly just below 2^32; 16 GiB of labels).  At beta =
    infinity a cold start is one cluster: Swendsen-Wang flips all or nothing by
    root 0's bit, Wolff flips all.  At beta = 0 every site is its own cluster:
    a Swendsen-Wang step flips site g iff its own flip bit is set (sampled rows
    against the contract's formula), and a Wolff step flips exactly its seed
    (the change of M and B equals that of flipping the seed alone)."""
    import torch
    P = _P()
    Lx, Ly = 65536, 65534
    N = Lx * Ly
    assert N < 2 ** 32
    b = P.Batch([dict(Lx=Lx, Ly=Ly, J=1.0, beta=math.inf, seed=6, replica=1, init=1)])
    sign = 1
    for t in range(2):
        b.cluster(1, "sw")
        B, M = b.observables()
        w = philox.philox4x32_10((0, t, 1, 8), philox.seed_key(6))
        if w[0] & 1:  # root 0: bit 0 of word 0
            sign = -sign
        assert M[0] == sign * N and B[0] == 2 * N
    b.cluster(1, "wolff")
    B, M = b.observables()
    assert M[0] == -sign * N and B[0] == 2 * N
    torch.cuda.synchronize()
    b.ws = None
    b.close()
    del b
    torch.cuda.empty_cache()

    b = P.Batch([dict(Lx=Lx, Ly=Ly, J=1.0, beta=0.0, seed=5, replica=0, init=0)])
    rows = [0, 1, 31, 32, 33, 40000, Ly - 2, Ly - 1]
    cols = list(range(0, 128)) + list(range(Lx - 128, Lx))
    full = b.get_spins(0)
    before = {y: full[y].copy() for y in rows}
    del full
    b.cluster(1, "sw")
    full = b.get_spins(0)
    key = philox.seed_key(5)
    for y in rows:
        for x in cols:
            gidx = y * Lx + x
            w = philox.philox4x32_10((gidx >> 7, 0, 0, 8), key)
            bit = (w[(gidx >> 5) & 3] >> (gidx & 31)) & 1
            assert full[y, x] == (-before[y][x] if bit else before[y][x]), (y, x)
    w = philox.philox4x32_10((0, 1, 0, 9), key)
    S = ((w[0] << 32) | w[1]) % N
    sy, sx = divmod(S, Lx)
    s_seed = int(full[sy, sx])
    nb = int(full[sy, (sx + 1) % Lx]) + int(full[sy, (sx - 1) % Lx]) + int(full[(sy + 1) % Ly, sx]) + \
        int(full[(sy - 1) % Ly, sx])
    del full
    B1, M1 = b.observables()
    b.cluster(1, "wolff")
    B2, M2 = b.observables()
    assert M2[0] - M1[0] == -2 * s_seed
    assert B2[0] - B1[0] == -2 * s_seed * nb
    torch.cuda.synchronize()
    b.ws = None
    b.close()
    del b
    torch.cuda.empty_cache()


def test_captured_chunks_record_across_replays():
    """40 SW steps (two replays of a captured 16-step chunk, then 8 direct
    steps) recorded every 3 steps, then 20 Wolff steps recorded every 5: the
    trace slots are computed on the device, so they continue across replays."""
    shapes = [(128, 66, 0.44, 31, 0), (64, 64, 0.3, 32, 0), (192, 34, 0.7, 33, 1)]
    g, o = _descs(shapes)
    P = _P()
    b = P.Batch(g)
    states = [oracle.init_state(d) for d in o]
    bond, mag = _gpu_cluster(b, 40, "sw", 3)
    ob, om = oracle.run_cluster_batch(o, states, 40, oracle.SWENDSEN_WANG, record_every=3)
    assert bond.shape == (3, 13)
    np.testing.assert_array_equal(bond, ob)
    np.testing.assert_array_equal(mag, om)
    bond, mag = _gpu_cluster(b, 20, "wolff", 5)
    ob, om = oracle.run_cluster_batch(o, states, 20, oracle.WOLFF, t0=40, record_every=5)
    np.testing.assert_array_equal(bond, ob)
    np.testing.assert_array_equal(mag, om)
    _check_states(b, states)
    b.close()


def test_graph_replays_between_eager_calls():
    """A captured chunk replayed several times with direct steps and sweeps
    in between; every stage against the oracle."""
    import torch
    shapes = [(64, 34, 0.44, 41, 0), (128, 8, 0.5, 42, 2)]
    g, o = _descs(shapes)
    P = _P()
    b = P.Batch(g)
    states = [oracle.init_state(d) for d in o]
    t = 0
    for rnd in range(3):
        _gpu_cluster(b, 16, "sw", 0)
        oracle.run_cluster_batch(o, states, 16, oracle.SWENDSEN_WANG, t0=t)
        t += 16
        _check_states(b, states)
        _gpu_cluster(b, 5, "sw", 0)
        oracle.run_cluster_batch(o, states, 5, oracle.SWENDSEN_WANG, t0=t)
        t += 5
        b.run(2)
        torch.cuda.synchronize()
        oracle.run_batch(o, states, 2, t0=t)
        t += 2
        _check_states(b, states)
    b.close()


def test_uneven_512_and_paper_scale_sampled():
    """Cluster steps of the uneven batch (512 replicas, 128^2 .. 8192^2; the
    tile lookup crosses replicas of every size) and of the paper-scale batch
    (754 x 512 x 528 cold starts, whose 528 rows leave a ragged 16-row tile,
    plus one 16384 x 12288 lattice): one replica of every size compared in full
    with the oracle, every replica's trace."""
    import workloads
    P = _P()
    for w, algo, n in ((workloads.uneven_512(), "sw", 3), (workloads.paper_scale(), "wolff", 2)):
        print(f"{w.name} {algo}", flush=True)
        g = [dict(Lx=r.Lx, Ly=r.Ly, J=r.J, beta=r.beta, seed=r.seed, replica=r.replica, init=r.init) for r in w.replicas]
        b = P.Batch(g)
        bond, mag = _gpu_cluster(b, n, algo, 1)
        seen, idx = set(), []
        for i, r in enumerate(w.replicas):
            if (r.Lx, r.Ly) not in seen:
                seen.add((r.Lx, r.Ly))
                idx.append(i)
        idx += [3, 100]  # two more replicas of common sizes
        o = [oracle.desc(w.replicas[i].Lx, w.replicas[i].Ly, w.replicas[i].J, w.replicas[i].beta,
                         w.replicas[i].seed, w.replicas[i].replica, w.replicas[i].init) for i in idx]
        states = [oracle.init_state(d) for d in o]
        ob, om = oracle.run_cluster_batch(o, states, n, ALGOS[algo], record_every=1)
        np.testing.assert_array_equal(bond[idx], ob)
        np.testing.assert_array_equal(mag[idx], om)
        for k, i in enumerate(idx):
            assert np.array_equal(b.get_spins(i), states[k]), (i, w.replicas[i].Lx, w.replicas[i].Ly)
        b.ws = None
        b.close()
