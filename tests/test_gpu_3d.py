"""Bit-exact parity of the 3D (simple cubic) sweeps of the HIP library,
through its C ABI, with the CPU oracle: states and (B, M) traces element by
element for single lattices of many shapes (one and several words per row,
every group width of the sweep kernel, Ly = 2 and Lz = 2 double bonds), the special temperatures, a batch of mixed
shapes, split runs, spin round trips, and the full-size benchmark batch on
sampled replicas; the largest lattice under exact properties."""
import math

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

# W = Lx / 64 words per row: odd widths take groups of 1 word, 2 mod 4 groups
# of 2, multiples of 4 groups of 4 (Ly = Lz = 2 double bonds, one and many
# groups per row, a row of one group, several workgroups with a partial last one)
SHAPES = [(64, 2, 2), (64, 4, 6), (128, 6, 4), (64, 64, 64), (192, 10, 14), (256, 2, 8), (64, 30, 2),
          (256, 2, 2), (256, 6, 10), (512, 4, 6), (768, 10, 4), (1024, 2, 2), (256, 64, 34)]


def _P():
    import paper_2404_16990_amd as P
    return P


def _descs(shapes, rng=0):
    """rng: 0 or 1 for every replica, or None to alternate the two contracts."""
    pick = (lambda i: i % 2) if rng is None else (lambda i: rng)
    g = [dict(Lx=Lx, Ly=Ly, Lz=Lz, J=1.0, beta=beta, seed=seed, replica=i, init=init, rng=pick(i))
         for i, (Lx, Ly, Lz, beta, seed, init) in enumerate(shapes)]
    o = [oracle.desc3(Lx, Ly, Lz, 1.0, beta, seed, i, init, rng=pick(i))
         for i, (Lx, Ly, Lz, beta, seed, init) in enumerate(shapes)]
    return g, o


def _run(b, n, every):
    import torch
    out = b.run(n, every)
    torch.cuda.synchronize()
    return (out[0].cpu().numpy(), out[1].cpu().numpy()) if out is not None else (None, None)


def _check_states(b, states):
    for i, s in enumerate(states):
        assert np.array_equal(b.get_spins(i), s), f"state mismatch in replica {i} {s.shape}"


def test_initial_states():
    g, o = _descs([(Lx, Ly, Lz, 0.2, 40 + i, i % 3) for i, (Lx, Ly, Lz) in enumerate(SHAPES)])
    b = _P().Batch3(g)
    _check_states(b, [oracle.init_state3(d) for d in o])
    B, M = b.observables()
    for i, d in enumerate(o):
        assert (B[i], M[i]) == oracle.observables3(oracle.init_state3(d))
    b.close()


@pytest.mark.parametrize("rng", [0, 1])
@pytest.mark.parametrize("beta", [0.1, 0.2216546, 0.3, 0.6])
def test_shapes_full_trace(beta, rng):
    print(f"3d beta={beta} rng={rng}", flush=True)
    g, o = _descs([(Lx, Ly, Lz, beta, 100 + i, 0) for i, (Lx, Ly, Lz) in enumerate(SHAPES)], rng)
    b = _P().Batch3(g)
    bond, mag = _run(b, 12, 1)
    states = [oracle.init_state3(d) for d in o]
    ob, om = oracle.run_batch3(o, states, 12, record_every=1)
    np.testing.assert_array_equal(bond, ob)
    np.testing.assert_array_equal(mag, om)
    _check_states(b, states)
    assert all(b.get_sweep(i) == 12 for i in range(len(g)))
    b.close()


@pytest.mark.parametrize("rng", [0, 1])
def test_special_temperatures(rng):
    shapes = [(64, 4, 4, 0.0, 7, 0), (128, 6, 2, math.inf, 8, 0), (64, 8, 8, math.inf, 9, 1),
              (64, 2, 2, math.inf, 10, 2), (64, 2, 2, 0.0, 11, 0), (256, 4, 2, 0.0, 12, 1), (512, 2, 4, math.inf, 13, 0)]
    g, o = _descs(shapes, rng)
    b = _P().Batch3(g)
    bond, mag = _run(b, 7, 1)
    states = [oracle.init_state3(d) for d in o]
    ob, om = oracle.run_batch3(o, states, 7, record_every=1)
    np.testing.assert_array_equal(bond, ob)
    np.testing.assert_array_equal(mag, om)
    _check_states(b, states)
    b.close()


def test_mixed_batch_split_runs_and_set_spins():
    rng = np.random.default_rng(3)
    shapes = [(int(64 * rng.choice([1, 2, 3, 4, 8])), int(2 * rng.integers(1, 12)), int(2 * rng.integers(1, 12)),
               float(1.0 / rng.uniform(3.0, 7.0)), 500 + i, int(rng.integers(0, 3))) for i in range(30)]
    g, o = _descs(shapes, None)  # the two random-number contracts alternate
    P = _P()
    b = P.Batch3(g)
    states = [oracle.init_state3(d) for d in o]
    _run(b, 5, 0)
    _run(b, 4, 0)
    oracle.run_batch3(o, states, 9)
    _check_states(b, states)
    # an arbitrary state written from the host, then more sweeps with recording
    s7 = np.where(rng.random(states[7].shape) < 0.3, 1, -1).astype(np.int8)
    b.set_spins(7, s7)
    states[7] = s7.copy()
    bond, mag = _run(b, 6, 3)
    ob, om = oracle.run_batch3(o, states, 6, t0=9, record_every=3)
    np.testing.assert_array_equal(bond, ob)
    np.testing.assert_array_equal(mag, om)
    _check_states(b, states)
    with pytest.raises(P.IsingError):
        b.set_spins(0, np.zeros(states[0].shape, dtype=np.int8))
    b.close()


@pytest.mark.parametrize("rng", [0, 1])
def test_benchmark_batch_sampled(rng):
    """The 3D benchmark batch (16 x 256^3, T from 3.5 to 5.5): 4 sweeps of the
    whole batch, three replicas compared in full with the oracle."""
    import workloads
    w = workloads.cubic_16x256()
    g = [dict(Lx=r.Lx, Ly=r.Ly, Lz=r.Lz, J=r.J, beta=r.beta, seed=r.seed, replica=r.replica, init=r.init, rng=rng)
         for r in w.replicas]
    b = _P().Batch3(g)
    bond, mag = _run(b, 4, 2)
    pick = [0, 7, 15]
    o = [oracle.desc3(w.replicas[i].Lx, w.replicas[i].Ly, w.replicas[i].Lz, w.replicas[i].J, w.replicas[i].beta,
                      w.replicas[i].seed, w.replicas[i].replica, w.replicas[i].init, rng=rng) for i in pick]
    states = [oracle.init_state3(d) for d in o]
    ob, om = oracle.run_batch3(o, states, 4, record_every=2)
    np.testing.assert_array_equal(bond[pick], ob)
    np.testing.assert_array_equal(mag[pick], om)
    for k, i in enumerate(pick):
        assert np.array_equal(b.get_spins(i), states[k]), i
    b.close()


def test_largest_lattice_exact_properties():
    """Lx*Ly*Lz just below 2^32 (2048 x 2048 x 1022): at beta = 0 a sweep
    negates the state (M -> -M, B kept); at beta = infinity a cold start is
    frozen."""
    import torch
    P = _P()
    Lx, Ly, Lz = 2048, 2048, 1022
    N = Lx * Ly * Lz
    assert N < 2 ** 32
    b = P.Batch3([dict(Lx=Lx, Ly=Ly, Lz=Lz, J=1.0, beta=0.0, seed=5, replica=0, init=0),
                  dict(Lx=Lx, Ly=Ly, Lz=Lz, J=1.0, beta=math.inf, seed=6, replica=1, init=1)])
    B0, M0 = b.observables()
    assert M0[1] == N and B0[1] == 3 * N and abs(M0[0]) < 10 * math.sqrt(N)
    b.run(1)
    B1, M1 = b.observables()
    assert M1[0] == -M0[0] and B1[0] == B0[0] and M1[1] == N and B1[1] == 3 * N
    b.run(1)
    B2, M2 = b.observables()
    assert M2[0] == M0[0] and B2[0] == B0[0]
    torch.cuda.synchronize()
    b.close()
    del b
    torch.cuda.empty_cache()
