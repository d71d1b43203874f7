"""The validation campaign of section 3.1 end to end on a small lattice:
validation.run_size on the GPU (an optional Swendsen-Wang burn-in of the
random starts, then Metropolis sweeps recorded every 10 sweeps, the batch's
schedule from the autotuner) against the oracle's own trajectories of the
same replicas bit for bit, the equilibration detection and averages of the
GPU traces equal to those of the oracle's traces, and the agreement summary
with the exact magnetisation below T_c once the starts are equilibrated."""
import math

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

TEMPS = [1.5, 2.0, 2.2, 2.6, 3.0, 3.5]


@pytest.mark.parametrize("rng,burnin", [(0, 0), (1, 25)])
def test_run_size_matches_the_oracle(rng, burnin):
    from paper_2404_16990_amd import validation
    L, sweeps, every, seed0 = 64, 2000, 10, 500
    res = validation.run_size(L, TEMPS, sweeps, every, rng, seed0=seed0, chunks=4, log=lambda s: None,
                              cluster_burnin=burnin, keep_traces=True)
    descs = [oracle.desc(L, L, 1.0, 1.0 / T, seed0 + i, i, oracle.INIT_RANDOM, rng=rng) for i, T in enumerate(TEMPS)]
    states = [oracle.init_state(d) for d in descs]
    if burnin:
        oracle.run_cluster_batch(descs, states, burnin, oracle.SWENDSEN_WANG)
    _, om = oracle.run_batch(descs, states, sweeps, t0=burnin, record_every=every)
    assert res["mag"].shape == (len(TEMPS), sweeps // every)
    assert np.array_equal(res["mag"], om)
    assert validation.analyse(om, TEMPS, L, every) == res["rows"]
    summary = validation.summarise(res)
    outside = [T for T in TEMPS if abs(T - validation.T_C) > 0.05]
    assert summary["checked"] == len(outside) and summary["agree"] + len(summary["misses"]) == len(outside)
    for r in res["rows"]:
        assert 0 <= r["t_eq_sweeps"] < sweeps and r["n_eff"] >= 1.0
        assert r["expected"] == validation.expected_m(r["T"], L)
    if burnin:
        # equilibrated starts: Yang's magnetisation well below T_c
        for r in res["rows"]:
            if r["T"] <= 2.0:
                assert abs(r["m"] - r["exact"]) < 0.01, r
                assert not any(math.isclose(mt[0], r["T"]) for mt in summary["misses"])
