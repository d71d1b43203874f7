"""Full-size, full-length runs of the benchmark configurations, checked against
exact results that hold at any size.

The oracle cannot replay 10^4 sweeps of 2.7e8 spins, so these runs are pinned
by physics instead: after equilibration the energy per spin of a replica away
from T_c equals Onsager's infinite-lattice value (finite-size corrections are
of order exp(-L / xi), far below the statistical errors at these sizes), and
|m| equals Yang's spontaneous magnetisation below T_c (cold starts, which need
no domain coarsening) or vanishes like N^-1/2 above it.  Means are taken over
the second half of each run, with errors from 10 bins.  The short-run bit
parity of the same configurations is in test_gpu_parity.py.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import exact, stats

pytestmark = pytest.mark.gpu


def _run(w, sweeps, every, idx=None):
    import torch
    import paper_2404_16990_amd as P
    descs = [dict(Lx=r.Lx, Ly=r.Ly, J=r.J, beta=r.beta, seed=r.seed, replica=r.replica, init=r.init)
             for r in w.replicas]
    b = P.Batch(descs)
    bond, mag = b.run(sweeps, every)
    torch.cuda.synchronize()
    n = np.array([r.Lx * r.Ly for r in w.replicas], dtype=np.float64)
    e = -bond.cpu().numpy().astype(np.float64) / n[:, None]
    m = mag.cpu().numpy().astype(np.float64) / n[:, None]
    b.close()
    return e, m


def _z(series, exact_value):
    half = series[series.size // 2:]
    mean, err = stats.binned_mean(half, nbins=10)
    return (mean - exact_value) / max(err, 1e-12), mean, err


def _check(w, e, m, above=2.45, below=None, max_z=5.0):
    checked = 0
    for r, rep in enumerate(w.replicas):
        T = rep.T
        if T >= above:
            z, mean, err = _z(e[r], exact.onsager_u(T))
            assert abs(z) < max_z, (r, T, mean, exact.onsager_u(T), err)
            # above T_c, <m^2> = chi / N with chi the sum of spin correlations; its
            # leading critical behaviour 0.9625 (1 - T_c/T)^(-7/4) bounds |m| with margin
            half = np.abs(m[r, m.shape[1] // 2:])
            chi = 0.9625 * (1.0 - exact.T_C / T) ** -1.75
            bound = 4.0 * math.sqrt(chi / (rep.Lx * rep.Ly))
            assert half.mean() < bound, (r, T, half.mean(), bound)
            checked += 1
        elif below is not None and T <= below:
            z, mean, err = _z(e[r], exact.onsager_u(T))
            assert abs(z) < max_z, (r, T, mean, exact.onsager_u(T), err)
            z, mean, err = _z(np.abs(m[r]), exact.yang_m(T))
            assert abs(z) < max_z, (r, T, mean, exact.yang_m(T), err)
            checked += 1
    return checked


def test_batch_256x1024_full_10k_sweeps_matches_onsager_above_tc():
    """Config of the benchmark: 256 x 1024^2, random starts, the full 10^4
    sweeps at the benchmark's recording cadence; the 64 replicas with T >= 3.0
    (equilibrated within a few hundred sweeps) against Onsager."""
    w = workloads.batch_256x1024()
    e, m = _run(w, w.sweeps, w.record_every)
    assert e.shape == (256, 100)
    assert _check(w, e, m, above=3.0) == 64


def test_uneven_512_full_2000_sweeps_matches_onsager_above_tc():
    """Uneven batch (128^2 ... 8192^2) for its full 2000 sweeps; every replica
    with T >= 2.45 (correlation length <= 8 sites) against Onsager."""
    w = workloads.uneven_512()
    e, m = _run(w, w.sweeps, 10)
    n = _check(w, e, m, above=2.45)
    assert n >= 100, n


def test_paper_scale_full_1000_sweeps_matches_onsager_and_yang():
    """754 x 512x528 cold starts (plus the 16384 x 12288 lattice) for the full
    1000 sweeps: energy against Onsager and |m| against Yang for T <= 2.05, and
    energy against Onsager for T >= 2.45.  The big lattice at T_c relaxes from
    the cold start towards the critical energy -sqrt(2) from below."""
    w = workloads.paper_scale()
    e, m = _run(w, w.sweeps, 5)
    n = _check(w, e, m, above=2.45, below=2.05)
    assert n >= 300, n
    big = e[-1]
    assert big[0] < big[-1] < -math.sqrt(2.0) + 0.02, (big[0], big[-1])
    assert np.all(np.diff(big[:20]) > 0)  # monotone relaxation early on


def test_largest_lattice_exact_properties():
    """The largest lattice the library accepts (Lx*Ly just below 2^32: 65536 x
    65534, 512 MiB of spins) under exact properties of the rule: at beta = 0
    every proposal is accepted, so a sweep flips every spin (M -> -M, B kept,
    and two sweeps restore the state); at beta = infinity a cold start is
    frozen (nothing with dE > 0 is accepted and no site has dE <= 0)."""
    import torch
    import paper_2404_16990_amd as P
    Lx, Ly = 65536, 65534
    assert Lx * Ly < 2**32
    for rng in (0, 1):
        b = P.Batch([dict(Lx=Lx, Ly=Ly, J=1.0, beta=0.0, seed=5, replica=0, init=0, rng=rng),
                     dict(Lx=Lx, Ly=Ly, J=1.0, beta=math.inf, seed=6, replica=1, init=1, rng=rng)])
        B0, M0 = b.observables()
        assert M0[1] == Lx * Ly and B0[1] == 2 * Lx * Ly
        assert B0[0] % 4 == (2 * Lx * Ly) % 4 and abs(M0[0]) < 10 * math.sqrt(Lx * Ly)
        b.run(1)
        B1, M1 = b.observables()
        assert M1[0] == -M0[0] and B1[0] == B0[0]
        assert M1[1] == M0[1] and B1[1] == B0[1]
        b.run(1)
        B2, M2 = b.observables()
        assert M2[0] == M0[0] and B2[0] == B0[0]
        torch.cuda.synchronize()
        b.close()
        del b
        torch.cuda.empty_cache()


def test_batch_256x1024_swendsen_wang_matches_onsager_and_yang():
    """Swendsen-Wang steps of the benchmark batch (256 x 1024^2, random
    starts).  Cluster steps equilibrate in a few dozen steps at every
    temperature, including below T_c where single-spin sweeps from a random
    start are stuck in domains, so 400 steps (the second half averaged) pin
    the energy to Onsager and |m| to Yang on both sides of T_c."""
    import torch
    import paper_2404_16990_amd as P
    w = workloads.batch_256x1024()
    b = P.Batch([dict(Lx=r.Lx, Ly=r.Ly, J=r.J, beta=r.beta, seed=r.seed, replica=r.replica, init=r.init)
                 for r in w.replicas])
    bond, mag = b.cluster(400, "sw", 1)
    torch.cuda.synchronize()
    n = float(1024 * 1024)
    e = -bond.cpu().numpy().astype(np.float64) / n
    m = mag.cpu().numpy().astype(np.float64) / n
    b.ws = None
    b.close()
    assert _check(w, e, m, above=2.45, below=2.15) >= 200


def test_cubic_series_on_the_gpu():
    """3D sweeps on 8 x 128 x 96 x 96 lattices against the high-temperature series
    <s s'> = t + 4 t^3 + O(t^5) at T = 12 and the low-temperature
    magnetisation 1 - 2 u^6 - 12 u^10 + O(u^12) of cold starts at T = 2."""
    import torch
    import paper_2404_16990_amd as P
    Lx, L = 128, 96
    hot = [dict(Lx=Lx, Ly=L, Lz=L, J=1.0, beta=1.0 / 12.0, seed=900 + r, replica=r, init=0) for r in range(8)]
    cold = [dict(Lx=Lx, Ly=L, Lz=L, J=1.0, beta=0.5, seed=950 + r, replica=8 + r, init=1) for r in range(8)]
    b = P.Batch3(hot + cold)
    bond, mag = b.run(600, 1)
    torch.cuda.synchronize()
    b.close()
    N = float(Lx * L * L)
    ss = bond.cpu().numpy()[:8, 100:].astype(np.float64) / (3 * N)
    per = ss.mean(axis=1)
    mean, err = per.mean(), per.std(ddof=1) / math.sqrt(8)
    t = math.tanh(1.0 / 12.0)
    assert abs(mean - (t + 4 * t ** 3)) < 40 * t ** 5 + 4 * err, (mean, t + 4 * t ** 3, err)
    mm = mag.cpu().numpy()[8:, 50:].astype(np.float64) / N
    per = mm.mean(axis=1)
    mean, err = per.mean(), per.std(ddof=1) / math.sqrt(8)
    u = math.exp(-1.0)
    series = 1 - 2 * u ** 6 - 12 * u ** 10
    assert abs(mean - series) < 20 * u ** 12 + 4 * err, (mean, series, err)
