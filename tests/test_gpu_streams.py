"""Batches on different HIP streams run concurrently and stay independent: two
2D batches and a 3D batch, each created on its own (default-priority) stream,
get Metropolis sweeps (graph-captured chunks and a remainder), cluster steps
and 3D sweeps enqueued interleaved with no synchronisation in between; each
batch's traces and final states must equal the oracle's for that batch alone.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def test_interleaved_batches_on_three_streams():
    import torch
    import paper_2404_16990_amd as P
    s1, s2, s3 = torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.Stream()
    d1 = [dict(Lx=256, Ly=130, J=1.0, beta=1 / 2.4, seed=11, replica=r, init=0) for r in range(6)]
    d2 = [dict(Lx=128 + 64 * (r % 3), Ly=2 + 16 * r, J=1.0, beta=0.3 + 0.1 * r, seed=22, replica=r, init=r % 3,
               rng=r % 2) for r in range(5)]
    d3 = [dict(Lx=128, Ly=10, Lz=6, J=1.0, beta=0.25, seed=33, replica=r, init=0, rng=r % 2) for r in range(3)]
    b1, b2, b3 = P.Batch(d1, stream=s1), P.Batch(d2, stream=s2), P.Batch3(d3, stream=s3)
    # enqueue everything before any synchronisation
    r1a = b1.run(37, 1)            # two graph chunks and a remainder at the default schedule
    r2a = b2.run(20, 4)
    r3a = b3.run(9, 3)
    r1b = b1.cluster(19, "sw", 1)  # a captured 16-step chunk and 3 direct steps
    r2b = b2.cluster(5, "wolff", 1)
    r3b = b3.run(4, 2)
    r1c = b1.run(5, 5)
    torch.cuda.synchronize()

    o1 = [oracle.desc(d["Lx"], d["Ly"], d["J"], d["beta"], d["seed"], d["replica"], d["init"]) for d in d1]
    o2 = [oracle.desc(d["Lx"], d["Ly"], d["J"], d["beta"], d["seed"], d["replica"], d["init"], rng=d["rng"])
          for d in d2]
    o3 = [oracle.desc3(d["Lx"], d["Ly"], d["Lz"], d["J"], d["beta"], d["seed"], d["replica"], d["init"], rng=d["rng"])
          for d in d3]
    st1 = [oracle.init_state(d) for d in o1]
    st2 = [oracle.init_state(d) for d in o2]
    st3 = [oracle.init_state3(d) for d in o3]
    want = [oracle.run_batch(o1, st1, 37, record_every=1),
            oracle.run_cluster_batch(o1, st1, 19, oracle.SWENDSEN_WANG, t0=37, record_every=1),
            oracle.run_batch(o1, st1, 5, t0=56, record_every=5),
            oracle.run_batch(o2, st2, 20, record_every=4),
            oracle.run_cluster_batch(o2, st2, 5, oracle.WOLFF, t0=20, record_every=1),
            oracle.run_batch3(o3, st3, 9, record_every=3),
            oracle.run_batch3(o3, st3, 4, t0=9, record_every=2)]
    got = [r1a, r1b, r1c, r2a, r2b, r3a, r3b]
    for k, ((gb, gm), (ob, om)) in enumerate(zip(got, want)):
        assert np.array_equal(gb.cpu().numpy(), ob) and np.array_equal(gm.cpu().numpy(), om), k
    for b, states in ((b1, st1), (b2, st2), (b3, st3)):
        for i, s in enumerate(states):
            assert np.array_equal(b.get_spins(i), s), i
    for b in (b1, b2, b3):
        b.close()
