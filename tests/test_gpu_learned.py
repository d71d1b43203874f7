"""Learned block proposals on the GPU, through the C ABI.

- the BF16 matrix-core lane layout the kernels assume;
- forward logits against the float64 reference evaluated at the same BF16
  rounding points; gradients against the exact float64 backward;
- the incremental pass: causal, sum_x q(x) = 1, scoring reproduces the
  sampler's own log q bit for bit, sampler frequencies match q;
- Metropolis-Hastings block rounds keep the Boltzmann distribution: mean
  energy against the exact transfer-matrix / Kaufman values, with untrained
  and trained networks, alone and interleaved with checkerboard sweeps;
- training lowers the loss and raises the block acceptance rate.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import exact, nn_ref, stats
import workloads

pytestmark = pytest.mark.gpu
C = 64


def _P():
    import paper_2404_16990_amd as P
    return P


def _dev(a, dtype):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _rand_blocks(rng, n, Bs):
    x = np.where(rng.random((n, Bs * Bs)) < 0.5, 1, -1).astype(np.int8)
    bnd = np.where(rng.random((n, 4 * Bs)) < 0.5, 1, -1).astype(np.int8)
    kc = rng.uniform(0.35, 0.55, size=n).astype(np.float32)
    return x, bnd, kc


def _params(scale=1.0, seed=16990):
    th = workloads.nn_initial_params(C, seed).astype(np.float64)
    return (th * scale).astype(np.float32)


def test_mfma_lane_layout():
    from paper_2404_16990_amd import probe
    assert probe.mfma_layout()


@pytest.mark.parametrize("Bs", [8, 4, 2])
def test_forward_matches_reference_at_bf16_points(Bs):
    import torch
    P = _P()
    rng = np.random.default_rng(Bs)
    theta = _params(1.5)
    x, bnd, kc = _rand_blocks(rng, 24, Bs)
    net = P.Net(theta, block=Bs, max_batch=64, max_seq=64)
    logits, _, loss = net.forward_backward(_dev(x, torch.int8), _dev(bnd, torch.int8), _dev(kc, torch.float32))
    torch.cuda.synchronize()
    g = logits.cpu().numpy().reshape(-1, Bs, Bs)
    ref, _ = nn_ref.forward(theta.astype(np.float64), C, x.reshape(-1, Bs, Bs), bnd, kc, bf16=True)
    # Only fp32 arithmetic (accumulation order, the exp2/rcp tanh, ~1e-7
    # absolute) differs from the reference here.  Where that moves an
    # activation across a bf16 rounding boundary the activation changes by one
    # bf16 ulp (<= 2^-8), i.e. a logit by ~2^-8 * |w| (|w| ~ 0.1) per crossing;
    # a few crossings can meet in one logit.  A systematic error would move
    # the mean deviation, which stays at fp32 level.
    dev = np.abs(g - ref)
    assert dev.max() < 5e-3 and dev.mean() < 3e-4, (dev.max(), dev.mean())
    exact_ref, _ = nn_ref.forward(theta.astype(np.float64), C, x.reshape(-1, Bs, Bs), bnd, kc)
    assert abs(float(loss.cpu()) - nn_ref.nll(exact_ref, x.reshape(-1, Bs, Bs))) < 5e-3


def test_gradient_matches_float64_backward():
    import torch
    P = _P()
    rng = np.random.default_rng(3)
    Bs = 8
    theta = _params(1.2)
    x, bnd, kc = _rand_blocks(rng, 48, Bs)
    net = P.Net(theta, block=Bs, max_batch=64, max_seq=64)
    _, grad, _ = net.forward_backward(_dev(x, torch.int8), _dev(bnd, torch.int8), _dev(kc, torch.float32))
    torch.cuda.synchronize()
    gg = grad.cpu().numpy().astype(np.float64)
    _, ref = nn_ref.loss_and_grad(theta.astype(np.float64), C, x.reshape(-1, Bs, Bs).astype(np.float64), bnd, kc)
    cos = float(gg @ ref / (np.linalg.norm(gg) * np.linalg.norm(ref)))
    rel = float(np.linalg.norm(gg - ref) / np.linalg.norm(ref))
    # BF16 operands (8 significant bits) in the forward and backward GEMMs
    assert cos > 0.999 and rel < 0.05, (cos, rel)
    # every parameter group gets a gradient of the right size
    Pg, Pr = nn_ref.unpack(gg, C), nn_ref.unpack(ref, C)
    for k in Pr:
        nr = np.linalg.norm(Pr[k])
        if nr > 1e-8:
            assert np.linalg.norm(Pg[k] - Pr[k]) / nr < 0.1, k


def test_q_sums_to_one_and_is_causal():
    import torch
    P = _P()
    Bs = 2
    theta = _params(2.0, seed=5)
    net = P.Net(theta, block=Bs, max_batch=16, max_seq=256)
    states = np.array(list(itertools.product([1, -1], repeat=4)), dtype=np.int8)
    rng = np.random.default_rng(9)
    for _ in range(4):
        bnd = np.where(rng.random(8) < 0.5, 1, -1).astype(np.int8)
        kc = np.float32(rng.uniform(0.3, 0.6))
        lq = net.score(_dev(states, torch.int8), _dev(np.tile(bnd, (16, 1)), torch.int8),
                       _dev(np.full(16, kc), torch.float32)).cpu().numpy()
        assert abs(np.exp(lq).sum() - 1.0) < 1e-12
        # the float64 reference at the same BF16 rounding points: only fp32 vs
        # fp64 arithmetic differs (sigmoid, tanh, accumulation order)
        for s, l in zip(states, lq):
            ref = nn_ref.log_q(theta.astype(np.float64), C, s.reshape(2, 2).astype(float), bnd, float(kc), bf16=True)
            assert abs(l - ref) < 1e-3, (l, ref)


@pytest.mark.parametrize("Bs", [8, 4, 2])
def test_scoring_reproduces_sampler_log_q_bitwise(Bs):
    import torch
    P = _P()
    rng = np.random.default_rng(Bs)
    net = P.Net(_params(1.0), block=Bs, max_batch=16, max_seq=512)
    _, bnd, kc = _rand_blocks(rng, 300, Bs)
    dbnd, dkc = _dev(bnd, torch.int8), _dev(kc, torch.float32)
    xs, lq = net.sample(dbnd, dkc, seed=77, replica=3, round_=5, blk0=1000)
    lq2 = net.score(xs, dbnd, dkc)
    assert torch.equal(lq, lq2)
    # another order and other neighbours in the workgroup: still identical
    perm = torch.tensor(rng.permutation(300), device="cuda")
    lq3 = net.score(xs[perm].contiguous(), dbnd[perm].contiguous(), dkc[perm].contiguous())
    assert torch.equal(lq3, lq2[perm])
    # the sampler is a pure function of (seed, replica, round, block id)
    xs2, lq4 = net.sample(dbnd, dkc, seed=77, replica=3, round_=5, blk0=1000)
    assert torch.equal(xs, xs2) and torch.equal(lq, lq4)


def test_sampler_frequencies_match_q():
    import torch
    P = _P()
    Bs, n = 2, 60000
    net = P.Net(_params(2.0, seed=8), block=Bs, max_batch=16, max_seq=n)
    bnd = np.array([1, -1, 1, 1, -1, -1, 1, -1], dtype=np.int8)
    xs, _ = net.sample(_dev(np.tile(bnd, (n, 1)), torch.int8), _dev(np.full(n, 0.44, np.float32), torch.float32),
                       seed=5, replica=0, round_=0)
    states = np.array(list(itertools.product([1, -1], repeat=4)), dtype=np.int8)
    idx = ((xs.cpu().numpy() < 0).astype(np.int64) * np.array([8, 4, 2, 1])).sum(axis=1)
    counts = np.bincount(idx, minlength=16)
    lq = net.score(_dev(states, torch.int8), _dev(np.tile(bnd, (16, 1)), torch.int8),
                   _dev(np.full(16, 0.44, np.float32), torch.float32)).cpu().numpy()
    _, _, p = stats.chi2_gof(counts, np.exp(lq) * n)
    assert p > 1e-3


# ---- Metropolis-Hastings block rounds keep the Boltzmann distribution -----------------

def _lnz_4x64(K):
    return exact.transfer_lnZ(4, 64, K)


def _moments_4x64(T):
    """Exact <B> and var(B) of the 64 x 4 torus from ln Z(K) (transfer matrix over 4-spin rows)."""
    K, h = 1.0 / T, 1e-4
    f0, fp, fm = _lnz_4x64(K), _lnz_4x64(K + h), _lnz_4x64(K - h)
    return (fp - fm) / (2 * h), (fp - 2 * f0 + fm) / (h * h)


def _run_blocks(P, Lx, Ly, Bs, T, R, theta, n_rounds, burn_sweeps, sweeps_between=0, seed0=4000):
    """Equilibrate with plain sweeps, then block rounds (and optional sweeps);
    returns per-replica bond sums B after every round and the acceptance rate."""
    import torch
    descs = [dict(Lx=Lx, Ly=Ly, J=1.0, beta=1.0 / T, seed=seed0 + r, replica=r, init=0) for r in range(R)]
    b = P.Batch(descs)
    b.run(burn_sweeps)
    net = P.Net(theta, block=Bs, max_batch=16, max_seq=8192)
    acc = torch.zeros(R, dtype=torch.int64, device="cuda")
    Bs_trace = []
    for m in range(n_rounds):
        b.block_round(net, m, acc)
        if sweeps_between:
            b.run(sweeps_between)
        B, _ = b.observables()
        Bs_trace.append(B.astype(np.float64))
    torch.cuda.synchronize()
    rate = float(acc.sum().cpu()) / (n_rounds * R * (Lx // Bs) * (Ly // Bs))
    return np.array(Bs_trace).T, rate


def _z(per_replica, target):
    m = per_replica.mean()
    return (m - target) / (per_replica.std(ddof=1) / math.sqrt(len(per_replica)))


@pytest.mark.parametrize("scale,sweeps", [(1.0, 0), (3.0, 0), (0.3, 0), (1.0, 1)])
def test_block_moves_keep_boltzmann_64x4(scale, sweeps):
    """Start in equilibrium (plain sweeps); Metropolis-Hastings block moves must
    keep the exact mean and variance of the bond sum."""
    P = _P()
    T = 2.5
    B, rate = _run_blocks(P, 64, 4, 2, T, 128, _params(scale, seed=21), 600, 400, sweeps)
    mean_B, var_B = _moments_4x64(T)
    assert rate > 0.01, rate  # the chains really move
    assert abs(_z(B.mean(axis=1), mean_B)) < 4, (B.mean(), mean_B, rate)
    # second moment around the exact mean
    assert abs(_z(((B - mean_B) ** 2).mean(axis=1), var_B)) < 4, (((B - mean_B) ** 2).mean(), var_B, rate)


def test_block_moves_8x8_keep_boltzmann_64x16():
    P = _P()
    T = 2.4
    B, rate = _run_blocks(P, 64, 16, 8, T, 96, _params(1.0, seed=22), 400, 400, 1)
    target = -exact.kaufman_energy(64, 16, T) * 64 * 16
    assert abs(_z(B.mean(axis=1), target)) < 4, (B.mean(), target, rate)


# ---- training: loss falls and block acceptance rises -----------------------------------

def test_training_reduces_loss_and_raises_acceptance():
    import torch
    from paper_2404_16990_amd import learned
    P = _P()
    Bs, T, R = 8, 2.3, 32
    descs = [dict(Lx=64, Ly=64, J=1.0, beta=1.0 / T, seed=900 + r, replica=r, init=0) for r in range(R)]
    b = P.Batch(descs)
    b.run(500)
    X, BN, K = learned.collect_blocks(b, Bs, 16, 20, 20)
    net = P.Net(_params(1.0), block=Bs, max_batch=512, max_seq=8192)
    untrained = P.Net(_params(1.0), block=Bs, max_batch=16, max_seq=8192)
    hist = learned.train(net, X, BN, K, 300, 512, 2e-3, seed=0, log_every=50)
    losses = [l for _, l in hist]
    assert losses[-1] < 0.8 * losses[0], losses
    # acceptance of block moves on the equilibrated lattices
    rates = {}
    for name, m in (("untrained", untrained), ("trained", net)):
        acc = torch.zeros(R, dtype=torch.int64, device="cuda")
        for r in range(10):
            b.block_round(m, 100 + r, acc)
        torch.cuda.synchronize()
        rates[name] = float(acc.sum()) / (10 * R * 64)
    assert rates["trained"] > 2 * rates["untrained"] + 0.01, rates


def test_sampled_minibatch_rows_follow_the_philox_definition():
    """train_step_sampled == train_step on the rows floor(u n / 2^32), u the
    first word of Philox(counter (i, k, 0, 6), key seed), for steps k = 0, 1, 2."""
    import torch
    from oracle import philox
    P = _P()
    rng = np.random.default_rng(77)
    Bs, n_rows, batch, seed = 4, 1000, 96, 0x1234_5678_9ABC
    x, bnd, kc = _rand_blocks(rng, n_rows, Bs)
    X, BN, K = _dev(x, torch.int8), _dev(bnd, torch.int8), _dev(kc, torch.float32)
    a = P.Net(_params(1.0), block=Bs, max_batch=batch, max_seq=64)
    b = P.Net(_params(1.0), block=Bs, max_batch=batch, max_seq=64)
    key = philox.seed_key(seed)
    for k in range(3):
        rows = np.array([(philox.philox4x32_10((i, k, 0, 6), key)[0] * n_rows) >> 32 for i in range(batch)])
        a.train_step_sampled(X, BN, K, batch, 1e-3, seed)
        b.train_step(_dev(x[rows], torch.int8), _dev(bnd[rows], torch.int8), _dev(kc[rows], torch.float32), 1e-3)
        torch.cuda.synchronize()
        assert np.array_equal(a.params, b.params), k
