"""Pins for the oracle's update rule, thresholds, initial states and observables.

Each test checks the oracle against something other than itself: closed forms,
brute force from the Hamiltonian (section 1), invariants of the checkerboard
dynamics (Supplementary algorithm S2) and exact symmetries.
"""
import math

import mpmath
import numpy as np
import pytest

import oracle
from oracle import exact
from oracle import philox as pyphilox
import workloads


# ---- thresholds (Metropolis rule, section 1) ---------------------------------

def test_thresholds_closed_form_at_exact_tc():
    # exp(-4 K_c) = (sqrt2 - 1)^2 = 3 - 2 sqrt2 and exp(-8 K_c) = 17 - 12 sqrt2
    thr4, thr8, always = oracle.thresholds(1.0, 1.0 / exact.T_C)
    with mpmath.workdps(50):
        e4 = (3 - 2 * mpmath.sqrt(2)) * 2**32
        e8 = (17 - 12 * mpmath.sqrt(2)) * 2**32
        # keep away from integer boundaries so a one-ulp libm difference cannot matter
        assert 0.01 < float(e4 - mpmath.floor(e4)) < 0.99
        assert 0.01 < float(e8 - mpmath.floor(e8)) < 0.99
        assert thr4 == int(mpmath.floor(e4)) == 736899888
        assert thr8 == int(mpmath.floor(e8)) == 126432032
    assert always == 0


@pytest.mark.parametrize("T", [0.5, 1.0, 2.269185, 3.0, 10.0, 1e6])
def test_thresholds_match_probability(T):
    thr4, thr8, _ = oracle.thresholds(1.0, 1.0 / T)
    with mpmath.workdps(40):
        for thr, de in ((thr4, 4), (thr8, 8)):
            p = mpmath.exp(-mpmath.mpf(de) / mpmath.mpf(T))
            # P(accept) = thr / 2^32 is p rounded down to the 2^-32 grid
            assert abs(mpmath.mpf(thr) / 2**32 - p) <= mpmath.mpf(2) ** -31


def test_thresholds_special_cases():
    assert oracle.thresholds(1.0, 0.0) == (0xFFFFFFFF, 0xFFFFFFFF, 1)
    assert oracle.thresholds(1.0, math.inf) == (0, 0, 0)
    # tiny K: p rounds to 1 in float64 -> clamp to 2^32 - 1, but not "always"
    assert oracle.thresholds(1.0, 1e-300)[2] == 0
    assert oracle.thresholds(1.0, 1e-300)[:2] == (0xFFFFFFFF, 0xFFFFFFFF)
    # J scales beta: (J, beta) and (2J, beta/2) agree
    assert oracle.thresholds(2.0, 0.25) == oracle.thresholds(1.0, 0.5)
    for J, beta in [(0.0, 1.0), (-1.0, 1.0), (math.inf, 1.0), (1.0, -0.1), (1.0, math.nan)]:
        with pytest.raises(ValueError):
            oracle.thresholds(J, beta)


# ---- brute force of one sweep from the Hamiltonian ---------------------------

def _energy(s, J):
    return -J * float((s * np.roll(s, -1, axis=1)).sum() + (s * np.roll(s, -1, axis=0)).sum())


def _brute_sweep(s, J, beta, seed, replica, t, rng=0):
    """One checkerboard sweep, every dE from H(s') - H(s) and the acceptance
    from exp(-beta dE) directly; the uniform for each site named through the
    pure-Python Philox with the contract's site mapping (rng 0) or the
    bit-sliced group words (rng 1)."""
    Ly, Lx = s.shape
    s = s.copy()
    for colour in (0, 1):
        for y in range(Ly):
            for x in range(Lx):
                if (x + y) & 1 != colour:
                    continue
                e0 = _energy(s, J)
                s[y, x] = -s[y, x]
                dE = _energy(s, J) - e0
                s[y, x] = -s[y, x]
                if dE <= 0 or beta * J == 0:
                    accept = True
                else:
                    uni = pyphilox.bitsliced_uniform if rng == 1 else pyphilox.sweep_uniform
                    r = uni(seed, replica, t, colour, Lx, x, y)
                    accept = r / 2**32 < math.exp(-beta * dE)
                if accept:
                    s[y, x] = -s[y, x]
    return s


@pytest.mark.parametrize("rng", [0, 1])
@pytest.mark.parametrize("Lx,Ly", [(2, 2), (4, 4), (6, 4), (4, 6), (8, 2), (2, 8), (128, 2)])
@pytest.mark.parametrize("T", [0.8, 2.269185, 4.0])
def test_sweep_matches_brute_force(Lx, Ly, T, rng):
    J = 1.0
    d = oracle.desc(Lx, Ly, J, 1.0 / T, seed=1234567 + Lx, replica=3, init=oracle.INIT_RANDOM, rng=rng)
    s = oracle.init_state(d)
    ref = s.copy()
    for t in range(6 if Lx * Ly <= 64 else 2):
        oracle.sweeps(d, s, 1, t0=t)
        ref = _brute_sweep(ref, J, 1.0 / T, d.seed, d.replica, t, rng)
        assert np.array_equal(s, ref), (t, s, ref)


def test_sweep_brute_force_coupling_not_one():
    J, beta = 0.7, 0.9
    d = oracle.desc(6, 4, J, beta, seed=99, replica=1)
    s = oracle.init_state(d)
    ref = s.copy()
    for t in range(5):
        oracle.sweeps(d, s, 1, t0=t)
        ref = _brute_sweep(ref, J, beta, 99, 1, t)
    assert np.array_equal(s, ref)


# ---- initial states ----------------------------------------------------------

def test_random_init_uses_contract_mapping():
    d = oracle.desc(8, 6, seed=2**40 + 17, replica=9)
    s = oracle.init_state(d)
    for y in range(6):
        for x in range(8):
            u = pyphilox.init_uniform(d.seed, 9, 8, x, y)
            assert s[y, x] == (1 if u >= 2**31 else -1)


def test_random_init_is_balanced_and_cold_modes():
    d = oracle.desc(256, 256, seed=5, replica=0)
    s = oracle.init_state(d)
    assert abs(int(s.sum())) < 4 * 256  # 4 sigma of a fair +-1 sum over 65536 sites
    assert (oracle.init_state(oracle.desc(64, 8, init=oracle.INIT_UP)) == 1).all()
    assert (oracle.init_state(oracle.desc(64, 8, init=oracle.INIT_DOWN)) == -1).all()


def test_invalid_descriptors():
    for args in [(5, 4), (4, 5), (0, 4), (4, 0)]:
        with pytest.raises(ValueError):
            oracle.init_state(oracle.desc(*args))


# ---- observables: closed forms ----------------------------------------------

@pytest.mark.parametrize("Lx,Ly", [(4, 4), (8, 6), (64, 2), (16, 32)])
def test_observables_closed_forms(Lx, Ly):
    N = Lx * Ly
    x = np.arange(Lx)[None, :]
    y = np.arange(Ly)[:, None]
    up = np.ones((Ly, Lx), np.int8)
    assert oracle.observables(up) == (2 * N, N)
    assert oracle.observables(-up) == (2 * N, -N)
    af = np.where((x + y) % 2 == 0, 1, -1).astype(np.int8)
    assert oracle.observables(af) == (-2 * N, 0)
    cols = np.broadcast_to(np.where(x % 2 == 0, 1, -1), (Ly, Lx)).astype(np.int8)
    assert oracle.observables(cols) == (0, 0)
    if Lx % 4 == 0:
        wide = np.broadcast_to(np.where((x // 2) % 2 == 0, 1, -1), (Ly, Lx)).astype(np.int8)
        assert oracle.observables(wide) == (N, 0)
    one = up.copy()
    one[1, 1] = -1  # one flipped spin breaks four bonds
    assert oracle.observables(one) == (2 * N - 8, N - 2)


def test_observables_brute_force_random():
    s = workloads.random_pm1((10, 12), seed=3)
    B = sum(int(s[y, x]) * (int(s[y, (x + 1) % 12]) + int(s[(y + 1) % 10, x]))
            for y in range(10) for x in range(12))
    assert oracle.observables(s) == (B, int(s.sum()))


# ---- closed-form trajectories ------------------------------------------------

def test_infinite_temperature_flips_everything():
    d = oracle.desc(64, 10, beta=0.0, seed=4)
    s = oracle.init_state(d)
    s0 = s.copy()
    B0, M0 = oracle.observables(s0)
    b, m = oracle.sweeps(d, s, 7, record_every=1)
    assert np.array_equal(s, -s0)  # odd number of sweeps
    assert (b == B0).all()
    assert list(m) == [(-M0 if i % 2 == 0 else M0) for i in range(7)]


def test_zero_temperature_cold_start_is_frozen():
    d = oracle.desc(64, 8, beta=math.inf, init=oracle.INIT_UP)
    s = oracle.init_state(d)
    b, m = oracle.sweeps(d, s, 5, record_every=1)
    assert (s == 1).all() and (b == 2 * 512).all() and (m == 512).all()


def test_zero_temperature_antiferromagnet_orders_in_one_sweep():
    Lx, Ly = 64, 6
    x = np.arange(Lx)[None, :]
    y = np.arange(Ly)[:, None]
    s = np.where((x + y) % 2 == 0, 1, -1).astype(np.int8)
    d = oracle.desc(Lx, Ly, beta=math.inf)
    b, m = oracle.sweeps(d, s, 3, record_every=1)
    # red sites see four opposite neighbours and flip; blue sites then see four
    # aligned neighbours and stay: all spins are -1 after the first sweep
    assert (s == -1).all()
    assert (b == 2 * Lx * Ly).all() and (m == -Lx * Ly).all()


@pytest.mark.parametrize("T", [1.0, 2.269185, 3.5])
def test_trace_invariants(T):
    d = oracle.desc(32, 16, beta=1 / T, seed=11, replica=2)
    s = oracle.init_state(d)
    b, m = oracle.sweeps(d, s, 200, record_every=1)
    N = 32 * 16
    assert ((b - 2 * N) % 4 == 0).all() and ((m - N) % 2 == 0).all()
    assert (np.abs(b) <= 2 * N).all() and (np.abs(m) <= N).all()


# ---- symmetries --------------------------------------------------------------

def test_global_flip_symmetry():
    d = oracle.desc(16, 12, beta=1 / 2.4, seed=77, replica=4)
    s = oracle.init_state(d)
    t = -s
    b1, m1 = oracle.sweeps(d, s, 40, record_every=1)
    b2, m2 = oracle.sweeps(d, t, 40, record_every=1)
    assert np.array_equal(t, -s) and np.array_equal(b1, b2) and np.array_equal(m1, -m2)


def test_split_runs_equal_one_run():
    d = oracle.desc(16, 8, beta=1 / 2.2, seed=8, replica=1)
    a = oracle.init_state(d)
    b = a.copy()
    oracle.sweeps(d, a, 30)
    oracle.sweeps(d, b, 13)
    oracle.sweeps(d, b, 17, t0=13)
    assert np.array_equal(a, b)


def test_record_every_and_threads_do_not_change_results():
    descs = [oracle.desc(16, 8, beta=1 / (1.5 + 0.2 * r), seed=100 + r, replica=r) for r in range(7)]
    st1 = [oracle.init_state(d) for d in descs]
    st2 = [s.copy() for s in st1]
    b1, m1 = oracle.run_batch(descs, st1, 20, record_every=1, threads=1)
    b2, m2 = oracle.run_batch(descs, st2, 20, record_every=5, threads=3)
    assert all(np.array_equal(x, y) for x, y in zip(st1, st2))
    assert np.array_equal(b1[:, 4::5], b2) and np.array_equal(m1[:, 4::5], m2)
    for r, d in enumerate(descs):
        s = oracle.init_state(d)
        b, m = oracle.sweeps(d, s, 20, record_every=1)
        assert np.array_equal(b, b1[r]) and np.array_equal(s, st1[r])


@pytest.mark.parametrize("rng", [0, 1])
def test_row_split_threads_do_not_change_results(rng):
    """One lattice whose colour phases are split over its rows on 2..64 threads
    (row counts that do not divide, one thread per row, more threads than rows)
    equals the single-thread sweep, traces included; run_batch's mix of
    row-split replicas and one-replica-per-thread replicas does too."""
    for Lx, Ly in ((24, 14), (64, 6), (10, 2)):
        d = oracle.desc(Lx, Ly, beta=1 / 2.4, seed=77, replica=3, rng=rng)
        ref = oracle.init_state(d)
        b0, m0 = oracle.sweeps(d, ref, 30, t0=5, record_every=3)
        for th in (2, 3, 5, 7, 64):
            s = oracle.init_state(d)
            b, m = oracle.sweeps_rows(d, s, 30, t0=5, record_every=3, threads=th)
            assert np.array_equal(s, ref) and np.array_equal(b, b0) and np.array_equal(m, m0), (Lx, Ly, th)
    descs = [oracle.desc(64, 64, beta=0.4, seed=5, replica=0, rng=rng)] + \
            [oracle.desc(8, 4, beta=0.5, seed=6 + r, replica=1 + r, rng=rng) for r in range(5)]
    for th in (4, 16):   # the 64 x 64 replica alone on all threads; then every replica row-split
        st1 = [oracle.init_state(d) for d in descs]
        st2 = [s.copy() for s in st1]
        b1, m1 = oracle.run_batch(descs, st1, 12, t0=[3, 0, 1, 2, 3, 4], record_every=4, threads=1)
        b2, m2 = oracle.run_batch(descs, st2, 12, t0=[3, 0, 1, 2, 3, 4], record_every=4, threads=th)
        assert all(np.array_equal(x, y) for x, y in zip(st1, st2))
        assert np.array_equal(b1, b2) and np.array_equal(m1, m2)


@pytest.mark.parametrize("rng,name", [(0, "oracle_single64.json"), (1, "oracle_single64_bitsliced.json")])
def test_oracle_golden_trace_single_64(rng, name):
    """Regression pin: the stored trace was written by a script that calls only the oracle."""
    import hashlib
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    with open(path) as f:
        g = json.load(f)
    w = workloads.single_64()
    r = w.replicas[0]
    d = oracle.desc(r.Lx, r.Ly, r.J, r.beta, r.seed, r.replica, r.init, rng=rng)
    s = oracle.init_state(d)
    assert hashlib.sha256(s.tobytes()).hexdigest() == g["init_sha256"]
    b, m = oracle.sweeps(d, s, w.sweeps, record_every=w.record_every)
    assert [int(v) for v in b] == g["bond"] and [int(v) for v in m] == g["mag"]
    assert hashlib.sha256(s.tobytes()).hexdigest() == g["final_sha256"]
