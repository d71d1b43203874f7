"""Pins of the cluster-step oracle (Swendsen-Wang, Wolff) against what the
algorithms' definitions and the exact solution fix, independently of the
oracle's own code:

- cluster labels against scipy's connected components of the same bond set,
  the bond occupancies drawn with the second (pure-Python) Philox;
- the special cases beta = 0 (no occupied bond: every site its own cluster)
  and beta = infinity (every aligned bond occupied), in closed form;
- the exact one-step transition kernel of the 2x2 torus, enumerated from the
  textbook definition of each algorithm (which is checked to leave the
  Boltzmann distribution invariant), against the oracle's one-step statistics;
- long-run averages against exact enumeration (4x2 states, 4x4 classes) and
  Kaufman's finite-torus energy (16x16 at T_c).
Seeds are fixed, so pass/fail is deterministic.
"""
import itertools
import math

import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

import oracle
from oracle import exact, philox, stats

SW, WOLFF = oracle.SWENDSEN_WANG, oracle.WOLFF


def _bond_list(Lx, Ly):
    """(owner, other, dir) of every bond: each site's right (dir 0) and down (dir 1) bond."""
    out = []
    for y in range(Ly):
        for x in range(Lx):
            g = y * Lx + x
            out.append((g, y * Lx + (x + 1) % Lx, 0))
            out.append((g, ((y + 1) % Ly) * Lx + x, 1))
    return out


def _occupied_py(d, s, t):
    """Occupied bonds of step t, from the contract's prose with the pure-Python Philox."""
    thr, none = oracle.bond_threshold(d.J, d.beta)
    flat = s.reshape(-1)
    key = philox.seed_key(d.seed)
    occ = []
    for g, h, k in _bond_list(d.Lx, d.Ly):
        if none or flat[g] != flat[h]:
            continue
        w = philox.philox4x32_10((g >> 1, t, d.replica, 7), key)[2 * (g & 1) + k]
        if w >= thr:
            occ.append((g, h))
    return occ


def _min_index_labels(n, edges):
    if edges:
        a, b = np.array(edges).T
    else:
        a = b = np.zeros(0, dtype=np.int64)
    A = coo_matrix((np.ones(len(a)), (a, b)), shape=(n, n))
    _, comp = connected_components(A, directed=False)
    root = np.full(comp.max() + 1, n, dtype=np.int64)
    np.minimum.at(root, comp, np.arange(n))
    return root[comp]


@pytest.mark.parametrize("Lx,Ly,beta", [(2, 2, 0.44), (4, 2, 0.3), (8, 6, 0.44), (16, 10, 0.6),
                                        (64, 4, 0.44), (6, 8, math.inf), (12, 4, 0.0), (10, 10, 2.0)])
def test_labels_are_scipy_components(Lx, Ly, beta):
    for t in (0, 5, 77):
        d = oracle.desc(Lx, Ly, 1.0, beta, seed=1000 + Lx + Ly, replica=3)
        s = oracle.init_state(d)
        lab = oracle.cluster_labels(d, s, t).reshape(-1).astype(np.int64)
        ref = _min_index_labels(Lx * Ly, _occupied_py(d, s, t))
        np.testing.assert_array_equal(lab, ref)


def _sw_flip_bit(d, root, t):
    w = philox.philox4x32_10((root >> 7, t, d.replica, 8), philox.seed_key(d.seed))
    return (w[(root >> 5) & 3] >> (root & 31)) & 1


def _wolff_seed_py(d, t):
    w = philox.philox4x32_10((0, t, d.replica, 9), philox.seed_key(d.seed))
    return ((w[0] << 32) | w[1]) % (d.Lx * d.Ly)


def test_beta_zero_every_site_is_its_own_cluster():
    d = oracle.desc(16, 6, 1.0, 0.0, seed=9, replica=2)
    for t in (0, 3):
        s = oracle.init_state(d)
        before = s.reshape(-1).copy()
        oracle.cluster_steps(d, s, 1, SW, t0=t)
        flips = np.array([_sw_flip_bit(d, g, t) for g in range(d.Lx * d.Ly)])
        np.testing.assert_array_equal(s.reshape(-1), before * (1 - 2 * flips))
        assert 0 < flips.sum() < flips.size
        s = oracle.init_state(d)
        oracle.cluster_steps(d, s, 1, WOLFF, t0=t)
        diff = np.flatnonzero(s.reshape(-1) != before)
        assert list(diff) == [_wolff_seed_py(d, t)] == [oracle.wolff_seed(d, t)]


def test_infinite_beta_cold_start_is_one_cluster():
    d = oracle.desc(8, 4, 1.0, math.inf, seed=5, init=oracle.INIT_UP)
    assert oracle.bond_threshold(1.0, math.inf) == (0, 0)
    for t in range(8):
        s = oracle.init_state(d)
        assert (oracle.cluster_labels(d, s, t) == 0).all()
        oracle.cluster_steps(d, s, 1, SW, t0=t)
        assert (s == (-1 if _sw_flip_bit(d, 0, t) else 1)).all()
        s = oracle.init_state(d)
        oracle.cluster_steps(d, s, 1, WOLFF, t0=t)
        assert (s == -1).all()


def test_wolff_flips_exactly_the_component_of_its_seed():
    d = oracle.desc(16, 12, 1.0, 0.44, seed=77, replica=1)
    for t in range(6):
        s = oracle.init_state(d)
        lab = oracle.cluster_labels(d, s, t).reshape(-1)
        before = s.reshape(-1).copy()
        oracle.cluster_steps(d, s, 1, WOLFF, t0=t)
        S = _wolff_seed_py(d, t)
        flipped = s.reshape(-1) != before
        np.testing.assert_array_equal(flipped, lab == lab[S])


# ---- exact transition kernel of the 2x2 torus ------------------------------

def _components_py(n, edges):
    parent = list(range(n))

    def find(a):
        while parent[a] != a:
            a = parent[a]
        return a
    for a, b in edges:
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[max(ra, rb)] = min(ra, rb)
    return [find(a) for a in range(n)]


def _exact_kernel(Lx, Ly, K, algorithm):
    """P[i, j] = probability that one step maps state i to state j (state bit
    g set <=> s_g = -1), from the definitions: every aligned bond occupied with
    p = 1 - exp(-2K); Swendsen-Wang flips each cluster with probability 1/2,
    Wolff flips the cluster of a uniformly chosen site."""
    n = Lx * Ly
    p = 1.0 - math.exp(-2.0 * K)
    bonds = _bond_list(Lx, Ly)
    P = np.zeros((1 << n, 1 << n))
    for i in range(1 << n):
        s = [1 - 2 * ((i >> g) & 1) for g in range(n)]
        aligned = [(g, h) for g, h, _ in bonds if s[g] == s[h]]
        for occ in itertools.product((0, 1), repeat=len(aligned)):
            k = sum(occ)
            w = p ** k * (1.0 - p) ** (len(aligned) - k)
            if w == 0.0:
                continue
            root = _components_py(n, [e for e, o in zip(aligned, occ) if o])
            roots = sorted(set(root))
            if algorithm == SW:
                for f in itertools.product((0, 1), repeat=len(roots)):
                    flip = dict(zip(roots, f))
                    j = i ^ sum(1 << g for g in range(n) if flip[root[g]])
                    P[i, j] += w / (1 << len(roots))
            else:
                for seed in range(n):
                    j = i ^ sum(1 << g for g in range(n) if root[g] == root[seed])
                    P[i, j] += w / n
    return P


def _boltzmann(Lx, Ly, K):
    n = Lx * Ly
    bonds = _bond_list(Lx, Ly)
    B = np.array([sum((1 - 2 * ((i >> g) & 1)) * (1 - 2 * ((i >> h) & 1)) for g, h, _ in bonds)
                  for i in range(1 << n)])
    w = np.exp(K * (B - B.max()))
    return w / w.sum()


@pytest.mark.parametrize("algorithm", [SW, WOLFF])
def test_exact_2x2_kernel_is_stationary(algorithm):
    K = 0.37
    P = _exact_kernel(2, 2, K, algorithm)
    np.testing.assert_allclose(P.sum(axis=1), 1.0, atol=1e-12)
    pi = _boltzmann(2, 2, K)
    np.testing.assert_allclose(pi @ P, pi, atol=1e-12)


@pytest.mark.parametrize("algorithm", [SW, WOLFF])
@pytest.mark.parametrize("start", [0b0000, 0b0110, 0b0001, 0b0011])
def test_2x2_one_step_statistics_match_the_exact_kernel(algorithm, start):
    K = 0.37
    P = _exact_kernel(2, 2, K, algorithm)
    R = 40000
    descs = [oracle.desc(2, 2, 1.0, K, seed=31 + start, replica=r) for r in range(R)]
    s0 = np.array([1 - 2 * ((start >> g) & 1) for g in range(4)], dtype=np.int8).reshape(2, 2)
    states = [s0.copy() for _ in range(R)]
    oracle.run_cluster_batch(descs, states, 1, algorithm, t0=11)
    idx = np.array([sum(1 << g for g in range(4) if st.reshape(-1)[g] < 0) for st in states])
    obs = np.bincount(idx, minlength=16)
    exp_counts = R * P[start]
    possible = exp_counts > 0
    assert (obs[~possible] == 0).all()
    chi2, dof, pval = stats.chi2_gof(obs[possible], exp_counts[possible])
    assert pval > 1e-3, (obs, exp_counts, chi2, dof)


# ---- long runs against exact results ---------------------------------------

@pytest.mark.parametrize("algorithm,T", [(SW, 1.8), (SW, exact.T_C), (WOLFF, exact.T_C), (SW, 3.5)])
def test_4x2_state_distribution(algorithm, T):
    """Final states of independent chains against the enumerated Boltzmann law
    (Lx = 4 has single horizontal bonds, Ly = 2 double vertical ones)."""
    R = 30000
    descs = [oracle.desc(4, 2, 1.0, 1.0 / T, seed=707, replica=r) for r in range(R)]
    states = [oracle.init_state(d) for d in descs]
    oracle.run_cluster_batch(descs, states, 20, algorithm)
    idx = np.array([sum(1 << g for g in range(8) if st.reshape(-1)[g] < 0) for st in states])
    obs = np.bincount(idx, minlength=256)
    chi2, dof, pval = stats.chi2_gof(obs, R * _boltzmann(4, 2, 1.0 / T))
    assert pval > 1e-3, (chi2, dof, pval)


@pytest.mark.parametrize("algorithm,T", [(SW, 1.5), (SW, exact.T_C), (WOLFF, exact.T_C), (SW, 3.5),
                                         (WOLFF, 3.5)])
def test_4x4_energy_magnetisation_classes(algorithm, T):
    R = 1 << 15
    descs = [oracle.desc(4, 4, 1.0, 1.0 / T, seed=4242 + algorithm, replica=r) for r in range(R)]
    states = [oracle.init_state(d) for d in descs]
    oracle.run_cluster_batch(descs, states, 30, algorithm)
    B = np.array([oracle.observables(s)[0] for s in states])
    M = np.array([int(s.sum()) for s in states])
    eB, eM = exact.enumerate_torus(4, 4)
    p = exact.boltzmann_weights(eB, T)
    keys = (eB + 64) * 64 + (eM + 32)
    uk, inv = np.unique(keys, return_inverse=True)
    expected = np.bincount(inv, weights=p) * R
    obs_keys = np.searchsorted(uk, (B + 64) * 64 + (M + 32))
    assert np.all(uk[obs_keys] == (B + 64) * 64 + (M + 32))
    obs = np.bincount(obs_keys, minlength=uk.size)
    chi2, dof, pval = stats.chi2_gof(obs, expected)
    assert pval > 1e-3, (chi2, dof, pval)


@pytest.mark.parametrize("algorithm,steps", [(SW, 3000), (WOLFF, 6000)])
def test_16x16_energy_at_tc_matches_kaufman(algorithm, steps):
    R, L = 32, 16
    descs = [oracle.desc(L, L, 1.0, 1.0 / exact.T_C, seed=16990 + algorithm, replica=r) for r in range(R)]
    states = [oracle.init_state(d) for d in descs]
    bond, _ = oracle.run_cluster_batch(descs, states, steps, algorithm, record_every=1)
    e = -bond[:, steps // 5:].astype(np.float64) / (L * L)
    per_rep = e.mean(axis=1)
    mean, err = per_rep.mean(), per_rep.std(ddof=1) / math.sqrt(R)
    ref = exact.kaufman_energy(L, L, exact.T_C)
    assert abs(ref - (-1.4530648528134769)) < 1e-12
    assert abs(mean - ref) < 4.0 * err, (mean, ref, err)
    assert err < 2e-3
