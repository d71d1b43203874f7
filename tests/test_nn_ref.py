"""Pins for the float64 reference of the block-proposal network.

- central finite differences pin the analytic backward pass;
- hand-computable parameter settings pin the forward pass (taps, boundary
  features, beta input, head);
- causality (logit k ignores sites >= k) and sum_x q(x) = 1 over every block
  configuration (2x2 and 3x3) pin the autoregressive factorisation;
- the site-by-site sampler's frequencies match q (chi-square).
"""
import itertools
import math

import numpy as np
import pytest

from oracle import nn_ref, stats
from oracle import philox as pyphilox
import workloads


def _rand_blocks(rng, N, Bs):
    x = np.where(rng.random((N, Bs, Bs)) < 0.5, 1.0, -1.0)
    bnd = np.where(rng.random((N, 4 * Bs)) < 0.5, 1.0, -1.0)
    beta = rng.uniform(0.3, 0.6, size=N)
    return x, bnd, beta


@pytest.mark.parametrize("Bs,C", [(4, 3), (3, 5), (8, 2)])
def test_backward_matches_finite_differences(Bs, C):
    rng = np.random.default_rng(Bs * 10 + C)
    theta = rng.normal(0, 0.7, size=nn_ref.param_count(C))
    x, bnd, beta = _rand_blocks(rng, 3, Bs)
    _, g = nn_ref.loss_and_grad(theta, C, x, bnd, beta)
    h = 1e-6
    idx = rng.choice(len(theta), size=min(len(theta), 60), replace=False)
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (nn_ref.loss_and_grad(tp, C, x, bnd, beta)[0] - nn_ref.loss_and_grad(tm, C, x, bnd, beta)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 + 1e-5 * abs(fd), (i, fd, g[i])


def test_forward_closed_form_left_neighbour_chain():
    # C = 1: only the (0,-1) tap of layer 1 and the centre taps of layers 2..4
    C, Bs, a = 1, 4, 0.8
    P = nn_ref.unpack(np.zeros(nn_ref.param_count(C)), C)
    theta = np.zeros(nn_ref.param_count(C))
    P = nn_ref.unpack(theta, C)
    P["W1"][3, 0] = a
    for l in (2, 3, 4):
        P[f"W{l}"][4, 0, 0] = 1.0
    P["wo"][0] = 1.0
    rng = np.random.default_rng(0)
    x, bnd, beta = _rand_blocks(rng, 2, Bs)
    logits, _ = nn_ref.forward(theta, C, x, bnd, beta)
    left = np.zeros_like(x)
    left[:, :, 1:] = x[:, :, :-1]
    expect = np.tanh(np.tanh(np.tanh(np.tanh(a * left))))
    assert np.allclose(logits, expect, atol=1e-15)


def test_forward_closed_form_boundary_beta_and_up_tap():
    C, Bs = 1, 3
    theta = np.zeros(nn_ref.param_count(C))
    P = nn_ref.unpack(theta, C)
    P["U1"][:, 0] = [1.0, 2.0, 4.0, 8.0]   # up, down, left, right
    P["W1"][1, 0] = 16.0 / 64             # (-1,0) tap
    P["v1"][0] = 0.5
    P["b1"][0] = -0.25
    for l in (2, 3, 4):
        P[f"W{l}"][4, 0, 0] = 1.0
    P["wo"][0], P["bo"][0] = 2.0, 0.1
    x = np.array([[[1, -1, 1], [-1, -1, 1], [1, 1, -1]]], dtype=float)
    bnd = np.array([[1, -1, 1, -1, -1, 1, 1, 1, -1, -1, 1, 1]], dtype=float)  # top, bottom, left, right
    beta = np.array([0.4])
    logits, _ = nn_ref.forward(theta, C, x, bnd, beta)
    for i in range(Bs):
        for j in range(Bs):
            pre = 0.5 * 0.4 - 0.25
            pre += 1.0 * (bnd[0, j] if i == 0 else 0) + 2.0 * (bnd[0, Bs + j] if i == Bs - 1 else 0)
            pre += 4.0 * (bnd[0, 2 * Bs + i] if j == 0 else 0) + 8.0 * (bnd[0, 3 * Bs + i] if j == Bs - 1 else 0)
            pre += 0.25 * (x[0, i - 1, j] if i > 0 else 0)
            v = pre
            for _ in range(4):
                v = math.tanh(v)
            assert abs(logits[0, i, j] - (2.0 * v + 0.1)) < 1e-14


@pytest.mark.parametrize("Bs", [2, 3, 4])
def test_causality(Bs):
    C = 3
    rng = np.random.default_rng(5)
    theta = rng.normal(0, 1.0, size=nn_ref.param_count(C))
    x, bnd, beta = _rand_blocks(rng, 1, Bs)
    base, _ = nn_ref.forward(theta, C, x, bnd, beta)
    for k in range(Bs * Bs):
        y = x.copy().reshape(1, -1)
        y[0, k:] = -y[0, k:]
        got, _ = nn_ref.forward(theta, C, y.reshape(1, Bs, Bs), bnd, beta)
        assert np.array_equal(got.reshape(-1)[:k + 1], base.reshape(-1)[:k + 1])


@pytest.mark.parametrize("Bs", [2, 3])
def test_q_sums_to_one(Bs):
    C = 4
    rng = np.random.default_rng(11)
    theta = rng.normal(0, 1.2, size=nn_ref.param_count(C))
    bnd = np.where(rng.random(4 * Bs) < 0.5, 1.0, -1.0)
    total = 0.0
    for bits in itertools.product([1.0, -1.0], repeat=Bs * Bs):
        total += math.exp(nn_ref.log_q(theta, C, np.array(bits).reshape(Bs, Bs), bnd, 0.44))
    assert abs(total - 1.0) < 1e-12


def test_sampler_frequencies_match_q():
    Bs, C, n = 2, 4, 6000
    rng = np.random.default_rng(2)
    theta = rng.normal(0, 1.0, size=nn_ref.param_count(C))
    bnd = np.array([1, -1, 1, 1, -1, -1, 1, -1], dtype=float)
    counts = np.zeros(16)
    states = list(itertools.product([1.0, -1.0], repeat=4))
    for s in range(n):
        u = pyphilox.philox4x32_10((s, 0, 7, 3), (123, 0))
        x = nn_ref.sample(theta, C, bnd, 0.44, u)
        counts[states.index(tuple(x.ravel()))] += 1
    q = np.array([math.exp(nn_ref.log_q(theta, C, np.array(st).reshape(2, 2), bnd, 0.44)) for st in states])
    _, _, p = stats.chi2_gof(counts, q * n)
    assert p > 1e-3


def test_initial_params_layout():
    C = 64
    th = workloads.nn_initial_params(C)
    assert th.dtype == np.float32 and len(th) == nn_ref.param_count(C) == 62337
    P = nn_ref.unpack(th.astype(np.float64), C)
    assert np.all(P["b2"] == 0) and abs(P["W3"].std() - 1 / math.sqrt(320)) < 0.005
