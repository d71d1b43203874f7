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


# ---- Adam (Kingma and Ba, 2015) ----------------------------------------------------------

def test_adam_two_steps_by_hand():
    """g = 2 then g = -1 from zero moments, lr 0.01, beta1 0.9, beta2 0.999, eps 1e-8:
    step 1: m = 0.2, v = 0.004, m/(1 - 0.9) = 2, v/(1 - 0.999) = 4, delta = 0.01 * 2 / (2 + 1e-8);
    step 2: m = 0.18 - 0.1 = 0.08, v = 0.003996 + 0.001 = 0.004996, m/0.19 = 8/19,
            v/0.001999 = 2.4992496248..., sqrt = 1.5809015228..., delta = 0.0026633703797568..."""
    th, m, v = nn_ref.adam_step(np.array([1.0]), np.array([2.0]), np.zeros(1), np.zeros(1), 1, 0.01)
    assert abs(m[0] - 0.2) < 1e-16 and abs(v[0] - 0.004) < 1e-17
    assert abs(th[0] - (1.0 - 0.0099999999500000002)) < 1e-15
    th, m, v = nn_ref.adam_step(th, np.array([-1.0]), m, v, 2, 0.01)
    assert abs(m[0] - 0.08) < 1e-16 and abs(v[0] - 0.004996) < 1e-17
    assert abs(th[0] - (1.0 - 0.0099999999500000002 - 0.0026633703797568640)) < 1e-15


def test_adam_matches_the_papers_efficient_form():
    """With eps = 0 Algorithm 1 equals the reordered form of section 2 of Kingma
    and Ba: alpha_t = lr sqrt(1 - b2^t) / (1 - b1^t), theta -= alpha_t m / sqrt(v)."""
    rng = np.random.default_rng(4)
    th = rng.normal(size=50)
    m, v = np.zeros(50), np.zeros(50)
    th2, m2, v2 = th.copy(), np.zeros(50), np.zeros(50)
    for t in range(1, 8):
        g = rng.normal(size=50) * 10 ** rng.uniform(-3, 1, size=50)
        th, m, v = nn_ref.adam_step(th, g, m, v, t, 0.003, eps=0.0)
        m2 = 0.9 * m2 + 0.1 * g
        v2 = 0.999 * v2 + 0.001 * g * g
        th2 = th2 - 0.003 * math.sqrt(1 - 0.999 ** t) / (1 - 0.9 ** t) * m2 / np.sqrt(v2)
        assert np.allclose(th, th2, rtol=0, atol=1e-13)


# ---- the backward at the BF16 rounding points of the matrix-core layers --------------------

def _torch_loss_bf16_points(theta, C, x, bnd, beta, rounding=True):
    """The network again, written with torch conv2d and autograd (CPU, float64):
    straight-through rounding of the layer-2..4 weights and inputs to bfloat16,
    and an identity whose backward rounds the product's gradient to bfloat16."""
    import torch

    def rnd(t):
        return t.float().to(torch.bfloat16).double() if rounding else t

    class STE(torch.autograd.Function):
        @staticmethod
        def forward(ctx, t):
            return rnd(t)

        @staticmethod
        def backward(ctx, g):
            return g

    class GradRound(torch.autograd.Function):
        @staticmethod
        def forward(ctx, t):
            return t.clone()

        @staticmethod
        def backward(ctx, g):
            return rnd(g)

    th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    o = 0

    def take(*shape):
        nonlocal o
        n = int(np.prod(shape))
        a = th[o:o + n].reshape(shape)
        o += n
        return a

    W1, U1, v1, b1 = take(4, C), take(4, C), take(C), take(C)
    Wl, bl = [], []
    for _ in range(3):
        Wl.append(take(5, C, C))
        bl.append(take(C))
    wo, bo = take(C), take(1)
    N, Bs, _ = x.shape
    xt = torch.tensor(x, dtype=torch.float64)[:, None]
    bt = torch.tensor(bnd, dtype=torch.float64)
    taps = [(-1, -1), (-1, 0), (-1, 1), (0, -1), (0, 0)]

    # the masked 3x3 kernel [out][in][di+1][dj+1] built with index_put, so autograd reaches the weights
    def masked_kernel(w, n_taps, cin):
        k = torch.zeros(C, cin, 3, 3, dtype=torch.float64)
        for t in range(n_taps):
            di, dj = taps[t]
            k = k.index_put((torch.arange(C)[:, None], torch.arange(cin)[None, :],
                             torch.tensor(di + 1), torch.tensor(dj + 1)), w[t].reshape(cin, C).T)
        return k

    pre = torch.nn.functional.conv2d(xt, masked_kernel(W1, 4, 1), padding=1)
    feat = torch.zeros(N, 4, Bs, Bs, dtype=torch.float64)
    feat[:, 0, 0, :] = bt[:, 0:Bs]
    feat[:, 1, Bs - 1, :] = bt[:, Bs:2 * Bs]
    feat[:, 2, :, 0] = bt[:, 2 * Bs:3 * Bs]
    feat[:, 3, :, Bs - 1] = bt[:, 3 * Bs:4 * Bs]
    pre = pre + torch.einsum("nfij,fc->ncij", feat, U1)
    pre = pre + torch.tensor(beta, dtype=torch.float64)[:, None, None, None] * v1[None, :, None, None]
    h = torch.tanh(pre + b1[None, :, None, None])
    for l in range(3):
        k = masked_kernel(STE.apply(Wl[l]), 5, C)
        pre = GradRound.apply(torch.nn.functional.conv2d(STE.apply(h), k, padding=1))
        h = torch.tanh(pre + bl[l][None, :, None, None])
    logits = torch.einsum("ncij,c->nij", h, wo) + bo
    loss = torch.nn.functional.softplus(-xt[:, 0] * logits).mean()
    loss.backward()
    return float(loss.detach()), th.grad.numpy()


@pytest.mark.parametrize("Bs,C,scale", [(4, 6, 0.8), (8, 8, 1.5), (3, 5, 1.0)])
def test_backward_at_bf16_points_matches_autograd(Bs, C, scale):
    rng = np.random.default_rng(Bs * 100 + C)
    theta = rng.normal(0, scale, size=nn_ref.param_count(C))
    x, bnd, beta = _rand_blocks(rng, 5, Bs)
    loss, g = nn_ref.loss_and_grad(theta, C, x, bnd, beta, bf16=True)
    tl, tg = _torch_loss_bf16_points(theta, C, x, bnd, beta)
    assert abs(loss - tl) < 1e-13
    assert np.allclose(g, tg, rtol=1e-9, atol=1e-13), np.abs(g - tg).max()
    # the rounding is real: the bf16-point gradient differs from the exact one (more for larger weights)
    _, ge = nn_ref.loss_and_grad(theta, C, x, bnd, beta)
    rel = np.linalg.norm(g - ge) / np.linalg.norm(ge)
    assert 1e-5 < rel < 0.25, rel


def test_autograd_network_equals_exact_backward_without_rounding():
    """The torch formulation with the roundings removed is the exact network:
    it reproduces the finite-difference-pinned float64 backward."""
    rng = np.random.default_rng(8)
    Bs, C = 4, 5
    theta = rng.normal(0, 1.0, size=nn_ref.param_count(C))
    x, bnd, beta = _rand_blocks(rng, 3, Bs)
    tl, tg = _torch_loss_bf16_points(theta, C, x, bnd, beta, rounding=False)
    loss, g = nn_ref.loss_and_grad(theta, C, x, bnd, beta)
    assert abs(loss - tl) < 1e-13 and np.allclose(g, tg, rtol=1e-10, atol=1e-14)


# ---- batched sampler and scorer ------------------------------------------------------------

def test_batched_sampler_and_scorer_equal_the_single_block_ones():
    Bs, C, N = 3, 4, 6
    rng = np.random.default_rng(21)
    theta = rng.normal(0, 1.0, size=nn_ref.param_count(C))
    _, bnd, beta = _rand_blocks(rng, N, Bs)
    u = rng.integers(0, 2 ** 32, size=(N, Bs * Bs), dtype=np.uint64)
    xs, thr = nn_ref.sample_batch(theta, C, bnd, beta, u)
    lq, _ = nn_ref.log_q_batch(theta, C, xs, bnd, beta)
    for n in range(N):
        x1 = nn_ref.sample(theta, C, bnd[n], beta[n], [int(v) for v in u[n]])
        assert np.array_equal(x1, xs[n])
        assert abs(nn_ref.log_q(theta, C, xs[n], bnd[n], beta[n]) - lq[n]) < 1e-12
        # thresholds recorded by the sampler are the scorer's thresholds of the drawn block
        _, lg = nn_ref.log_q_batch(theta, C, xs[n:n + 1], bnd[n:n + 1], beta[n:n + 1])
        assert [nn_ref.threshold(v) for v in lg.ravel()] == [int(t) for t in thr[n]]
