"""Learned block proposals on the GPU, through the C ABI.

- the BF16 matrix-core lane layout the kernels assume;
- forward logits and gradients, element by element, against the float64
  reference evaluated at the same BF16 rounding points;
- Adam steps against a float64 Adam step fed the GPU's own gradient;
- training blocks extracted from the lattice against their definition (Philox
  positions, periodic boundary strips), bit for bit;
- the incremental pass at block sizes 8 and 4: log q and the sampled sites
  against the float64 network, causal, sum_x q(x) = 1, scoring reproduces
  the sampler's own log q bit for bit, sampler frequencies match q;
- Metropolis-Hastings block rounds keep the Boltzmann distribution: mean
  energy against the exact transfer-matrix / Kaufman values, with untrained
  and trained networks, alone and interleaved with checkerboard sweeps, and
  at the benchmark's shape (256^2, 8 x 8 blocks, trained network) against
  Kaufman's 256^2 energy with independent-replica errors;
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
    assert probe.mfma_layout_f32()


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


@pytest.mark.parametrize("Bs,n", [(8, 48), (4, 23), (2, 47)])
def test_gradient_matches_float64_backward_at_bf16_points(Bs, n):
    """Gradient element by element against the float64 backward evaluated at the
    kernels' bfloat16 rounding points (weights and inputs of the layer-2..4
    products, and the pre-activation gradients entering the backward
    products).  Only fp32 arithmetic differs, so the bound is cosine >= 0.9999
    and max |error| <= 1e-2 of the largest gradient, in every parameter group;
    per element, |error| <= 2e-2 |g| + 1e-3 of the group's largest entry (one
    bfloat16 rounding flip, 2^-8 relative, moves a product's contribution by
    less than that).  A 64-position tile holds 1, 4 or 16 blocks; 23 and 47
    blocks leave the last tile partly empty."""
    import torch
    P = _P()
    rng = np.random.default_rng(3 + Bs)
    theta = _params(1.2)
    x, bnd, kc = _rand_blocks(rng, n, Bs)
    net = P.Net(theta, block=Bs, max_batch=64, max_seq=64)
    _, grad, _ = net.forward_backward(_dev(x, torch.int8), _dev(bnd, torch.int8), _dev(kc, torch.float32))
    torch.cuda.synchronize()
    gg = grad.cpu().numpy().astype(np.float64)
    xb = x.reshape(-1, Bs, Bs).astype(np.float64)
    _, ref = nn_ref.loss_and_grad(theta.astype(np.float64), C, xb, bnd, kc, bf16=True)
    cos = float(gg @ ref / (np.linalg.norm(gg) * np.linalg.norm(ref)))
    nmax = float(np.abs(gg - ref).max() / np.abs(ref).max())
    print(f"gradient vs bf16-point reference: cos {cos:.8f}, normalised max error {nmax:.2e}")
    assert cos >= 0.9999 and nmax <= 1e-2, (cos, nmax)
    Pg, Pr = nn_ref.unpack(gg, C), nn_ref.unpack(ref, C)
    for k in Pr:
        scale = np.abs(Pr[k]).max()
        if scale < 1e-12:
            continue
        err = np.abs(Pg[k] - Pr[k])
        assert err.max() <= 1e-2 * scale, (k, err.max() / scale)
        bad = err > 2e-2 * np.abs(Pr[k]) + 1e-3 * scale
        assert not bad.any(), (k, int(bad.sum()), float((err / scale).max()))
    # the exact float64 backward is close as well (BF16 operands: 8 significant bits)
    _, exact_ref = nn_ref.loss_and_grad(theta.astype(np.float64), C, xb, bnd, kc)
    cos_e = float(gg @ exact_ref / (np.linalg.norm(gg) * np.linalg.norm(exact_ref)))
    assert cos_e > 0.999, cos_e


def test_adam_steps_match_float64_adam():
    """Four training steps: each step's parameters equal one float64 Adam step
    (Kingma and Ba, 2015; beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected)
    applied to the previous reference parameters with the gradient the GPU
    computed for that step, to fp32 rounding (a few ulps of the parameter plus
    1e-5 of the step size per step)."""
    import torch
    P = _P()
    rng = np.random.default_rng(31)
    Bs, lr = 8, 2e-3
    theta0 = _params(1.0)
    net = P.Net(theta0, block=Bs, max_batch=64, max_seq=64)
    th = theta0.astype(np.float64)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    for t in range(1, 5):
        x, bnd, kc = _rand_blocks(rng, 40, Bs)
        X, BN, K = _dev(x, torch.int8), _dev(bnd, torch.int8), _dev(kc, torch.float32)
        _, grad, _ = net.forward_backward(X, BN, K)
        g = grad.cpu().numpy().astype(np.float64)   # the gradient the step itself recomputes (deterministic)
        net.train_step(X, BN, K, lr)
        torch.cuda.synchronize()
        th, m, v = nn_ref.adam_step(th, g, m, v, t, lr)
        got = net.params.astype(np.float64)
        tol = t * (4 * np.spacing(np.abs(th).astype(np.float32)).astype(np.float64) + 1e-5 * lr)
        err = np.abs(got - th)
        assert np.all(err <= tol), (t, int((err > tol).sum()), float((err / tol).max()))
        # the step really moved every parameter with a nonzero gradient by ~lr
        moved = np.abs(got - theta0.astype(np.float64)) if t == 1 else None
        if t == 1:
            nz = np.abs(g) > 1e-6
            assert np.all(moved[nz] > 0.5 * lr), float(moved[nz].min())


def test_extract_blocks_follow_their_definition():
    """Training blocks: sample i of replica r sits at bx = w0 mod Lx/Bs,
    by = w1 mod Ly/Bs with (w0, w1, ...) = Philox(ctr = {i, draw, replica, 5},
    key = seed); block spins, the four boundary strips and K = beta*J are read
    from the lattice itself (get_spins), with periodic wrap."""
    import torch
    from oracle import philox
    P = _P()
    Lx, Ly, R = 128, 48, 3
    descs = [dict(Lx=Lx, Ly=Ly, J=1.0 + 0.25 * r, beta=0.41 + 0.02 * r, seed=0xFEED0000 + 977 * r, replica=5 + r,
                  init=0) for r in range(R)]
    b = P.Batch(descs)
    b.run(7)
    spins = [b.get_spins(r).astype(np.int8) for r in range(R)]
    for Bs, per, draw in ((8, 60, 3), (4, 50, 0xFFFFFFFF), (2, 40, 17)):
        blocks, bnd, coup = b.extract_blocks(Bs, per, draw)
        torch.cuda.synchronize()
        blocks, bnd, coup = blocks.cpu().numpy(), bnd.cpu().numpy(), coup.cpu().numpy()
        edges = set()
        for q in range(R * per):
            r, i = divmod(q, per)
            d = descs[r]
            o = philox.philox4x32_10((i, draw, d["replica"], 5), philox.seed_key(d["seed"]))
            bx, by = o[0] % (Lx // Bs), o[1] % (Ly // Bs)
            x0, y0 = bx * Bs, by * Bs
            s = spins[r]
            assert np.array_equal(blocks[q], s[y0:y0 + Bs, x0:x0 + Bs].ravel()), (Bs, q)
            expect = np.concatenate([s[(y0 - 1) % Ly, x0:x0 + Bs], s[(y0 + Bs) % Ly, x0:x0 + Bs],
                                     s[y0:y0 + Bs, (x0 - 1) % Lx], s[y0:y0 + Bs, (x0 + Bs) % Lx]])
            assert np.array_equal(bnd[q], expect), (Bs, q)
            assert coup[q] == np.float32(d["beta"] * d["J"]), (Bs, q)
            edges.add((bx == 0, by == 0, bx == Lx // Bs - 1, by == Ly // Bs - 1))
        assert len(edges) > 2  # wrapped boundaries were among the draws


@pytest.mark.parametrize("Bs", [8, 4, 2])
def test_sampler_and_scorer_match_the_float64_network(Bs):
    """The incremental kernels at the production block sizes against the float64
    network at the same bfloat16 rounding points.  log q is a sum of Bs^2 terms
    log sigmoid(+-logit), each moving by at most |d logit| (slope <= 1), so the
    forward bound on logits (5e-3 max, 3e-4 mean) gives |d log q| <= Bs^2 * 5e-3
    and a mean <= Bs^2 * 3e-4.  The sampler, fed the uniforms of its definition,
    draws the reference's sites until the first site whose uniform lies within
    2^32 * sigmoid' * 5e-3 <= 2^32 * 1.25e-3 of the reference threshold."""
    import torch
    from oracle import philox
    P = _P()
    rng = np.random.default_rng(40 + Bs)
    theta = _params(1.5, seed=41)
    th64 = theta.astype(np.float64)
    n, BB = 64, Bs * Bs
    _, bnd, kc = _rand_blocks(rng, n, Bs)
    net = P.Net(theta, block=Bs, max_batch=16, max_seq=n)
    dbnd, dkc = _dev(bnd, torch.int8), _dev(kc, torch.float32)
    seed, replica, round_, blk0 = 0xABCDEF012345, 7, 11, 300
    xs, lq = net.sample(dbnd, dkc, seed=seed, replica=replica, round_=round_, blk0=blk0)
    xr = np.where(rng.random((n, BB)) < 0.5, 1, -1).astype(np.int8)
    lq_r = net.score(_dev(xr, torch.int8), dbnd, dkc)
    torch.cuda.synchronize()
    xs, lq, lq_r = xs.cpu().numpy(), lq.cpu().numpy(), lq_r.cpu().numpy()
    # log q of the sampled blocks and of random blocks
    for blocks, got in ((xs, lq), (xr, lq_r)):
        ref, _ = nn_ref.log_q_batch(th64, C, blocks.reshape(n, Bs, Bs).astype(np.float64), bnd, kc, bf16=True)
        d = np.abs(got - ref)
        assert d.max() <= BB * 5e-3 and d.mean() <= BB * 3e-4, (d.max(), d.mean())
    # sampled sites against the reference sampler with the same uniforms
    key = philox.seed_key(seed)
    u = np.zeros((n, BB), dtype=np.uint64)
    for i in range(n):
        for k in range(BB):
            s = (blk0 + i) * BB + k
            u[i, k] = philox.philox4x32_10((s >> 2, round_, replica, 3), key)[s & 3]
    rx, rthr = nn_ref.sample_batch(th64, C, bnd, kc, u, bf16=True)
    margin = 2.0 ** 32 * 1.25e-3
    identical = 0
    for i in range(n):
        diff = np.nonzero(xs[i] != rx[i].ravel())[0]
        if len(diff) == 0:
            identical += 1
            continue
        k = diff[0]
        assert abs(float(u[i, k]) - float(rthr[i, k])) < margin, (i, k, int(u[i, k]), int(rthr[i, k]))
    assert identical >= n // 2, identical


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


def test_block_moves_exact_at_the_production_shape():
    """The benchmark's learned path on 256^2 lattices with 8 x 8 blocks and a
    network trained on the plain sampler's blocks: 48 independent replicas at
    T = 2.3 (distinct seeds), equilibrated by Swendsen-Wang steps, then units
    of one block round (both block colours) and one checkerboard sweep.  The
    mean energy per spin over the replicas' run means must equal Kaufman's
    exact value for the 256 x 256 torus within 4 standard errors of the
    spread between independent replicas (an error estimate that needs no
    autocorrelation time), and the blocks must really move."""
    import torch
    from paper_2404_16990_amd import learned
    P = _P()
    R, L, T = 48, 256, 2.3
    descs = [dict(Lx=L, Ly=L, J=1.0, beta=1.0 / T, seed=31000 + r, replica=r, init=0) for r in range(R)]
    b = P.Batch(descs)
    b.cluster(150, "sw")
    b.run(200)
    X, BN, K = learned.collect_blocks(b, 8, 16, 24, 25)
    net = P.Net(workloads.nn_initial_params(C), block=8, max_batch=512, max_seq=65536)
    hist = learned.train(net, X, BN, K, 400, 512, 2e-3, seed=3, log_every=100)
    assert hist[-1][1] < 0.8 * hist[0][1], hist
    acc = torch.zeros(R, dtype=torch.int64, device="cuda")
    _, e, _ = learned.unit_traces(b, 400, learned.learned_units(b, net, 0, acc))
    rate = float(acc.sum().cpu()) / (400 * R * (L // 8) ** 2)
    assert rate > 0.2, rate
    means = e[:, 50:].mean(axis=1)
    exact_e = exact.kaufman_energy(L, L, T)
    z = (means.mean() - exact_e) / (means.std(ddof=1) / math.sqrt(R))
    print(f"256^2 learned chain at T = {T}: <e> = {means.mean():.6f} +- {means.std(ddof=1) / math.sqrt(R):.6f}, "
          f"exact {exact_e:.6f}, z = {z:.2f}, block acceptance {rate:.3f}")
    assert abs(z) < 4, (means.mean(), exact_e, z)


def test_training_steps_replay_one_captured_graph():
    """40 sampled training steps with the same arguments replay one captured
    step (its step number lives on the device); setting the parameters
    restarts the count, so the same 40 steps again give the same parameters
    bit for bit."""
    import torch
    P = _P()
    rng = np.random.default_rng(12)
    Bs, batch = 4, 128
    x, bnd, kc = _rand_blocks(rng, 2000, Bs)
    X, BN, K = _dev(x, torch.int8), _dev(bnd, torch.int8), _dev(kc, torch.float32)
    theta0 = _params(1.0)
    net = P.Net(theta0, block=Bs, max_batch=batch, max_seq=64)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    for _ in range(40):
        net.train_step_sampled(X, BN, K, batch, 1e-3, 7, loss)
    torch.cuda.synchronize()
    a = net.params
    assert net.graph_stats() == (1, 1)
    assert not np.array_equal(a, theta0)
    net.set_params(theta0)
    for _ in range(40):
        net.train_step_sampled(X, BN, K, batch, 1e-3, 7, loss)
    torch.cuda.synchronize()
    assert np.array_equal(net.params, a)
    assert net.graph_stats() == (1, 1)


def test_multi_step_training_equals_single_steps():
    """train_steps_sampled(n) is n single sampled steps: 37 steps in one call
    (two replays of a captured 16-step graph, then a 5-step graph) leave the
    parameters and the last loss bit for bit where 37 single calls leave
    them."""
    import torch
    P = _P()
    rng = np.random.default_rng(13)
    Bs, batch = 8, 96
    x, bnd, kc = _rand_blocks(rng, 700, Bs)
    X, BN, K = _dev(x, torch.int8), _dev(bnd, torch.int8), _dev(kc, torch.float32)
    theta0 = _params(1.0)
    a = P.Net(theta0, block=Bs, max_batch=batch, max_seq=64)
    b = P.Net(theta0, block=Bs, max_batch=batch, max_seq=64)
    la = torch.zeros(1, dtype=torch.float32, device="cuda")
    lb = torch.zeros(1, dtype=torch.float32, device="cuda")
    a.train_steps_sampled(X, BN, K, batch, 2e-3, 5, 37, la)
    for _ in range(37):
        b.train_step_sampled(X, BN, K, batch, 2e-3, 5, lb)
    torch.cuda.synchronize()
    assert np.array_equal(a.params, b.params)
    assert float(la.cpu()) == float(lb.cpu())
    assert a.graph_stats() == (2, 2)
    assert not np.array_equal(a.params, theta0)


def _host_block_round(net, spins, descs, Bs, round_):
    """One block round computed on the host from its definition, with the
    library's standalone passes supplying the proposals and log q: colour 0
    (bx + by even) then colour 1 on the lattice colour 0 left; per block the
    current spins and boundary from the host lattice, the proposal from the
    sampler with the block's id and the round, log q of the current spins
    from the scorer, dB exactly, log A = K dB + log q(s) - log q(s'), and the
    53-bit uniform of Philox(counter (block id, round, replica, 4), key seed).
    Returns the new lattices, accepts per replica and the smallest
    |u - exp(log A)| met (a decision closer than FP64 rounding is undecided)."""
    import torch
    from oracle import philox
    out = [s.copy() for s in spins]
    acc = np.zeros(len(descs), dtype=np.int64)
    closest = 1.0
    for r, d in enumerate(descs):
        s = out[r]
        Ly, Lx = s.shape
        nbx, nby = Lx // Bs, Ly // Bs
        K = d["beta"] * d["J"]
        for colour in (0, 1):
            for by in range(nby):
                for bx in range(nbx):
                    if (bx + by) % 2 != colour:
                        continue
                    y0, x0 = by * Bs, bx * Bs
                    cur = s[y0:y0 + Bs, x0:x0 + Bs].copy()
                    bnd = np.concatenate([s[(y0 - 1) % Ly, x0:x0 + Bs], s[(y0 + Bs) % Ly, x0:x0 + Bs],
                                          s[y0:y0 + Bs, (x0 - 1) % Lx], s[y0:y0 + Bs, (x0 + Bs) % Lx]])
                    blk = by * nbx + bx
                    kc = np.array([K], dtype=np.float32)
                    prop, lq_p = net.sample(_dev(bnd[None], torch.int8), _dev(kc, torch.float32), d["seed"],
                                            d["replica"], round_, blk)
                    lq_c = net.score(_dev(cur.reshape(1, -1), torch.int8), _dev(bnd[None], torch.int8),
                                     _dev(kc, torch.float32))
                    prop = prop.cpu().numpy().reshape(Bs, Bs).astype(np.int64)
                    lq_p, lq_c = float(lq_p.cpu()[0]), float(lq_c.cpu()[0])

                    def bonds(x):
                        x = x.astype(np.int64)
                        inner = (x[:, :-1] * x[:, 1:]).sum() + (x[:-1, :] * x[1:, :]).sum()
                        edge = (x[0] * bnd[:Bs]).sum() + (x[-1] * bnd[Bs:2 * Bs]).sum() \
                            + (x[:, 0] * bnd[2 * Bs:3 * Bs]).sum() + (x[:, -1] * bnd[3 * Bs:]).sum()
                        return int(inner + edge)

                    log_a = K * (bonds(prop) - bonds(cur)) + lq_c - lq_p
                    o = philox.philox4x32_10((blk, round_, d["replica"], 4), philox.seed_key(d["seed"]))
                    u = float((int(o[0]) << 21) | (int(o[1]) >> 11)) * 2.0 ** -53
                    if log_a < 0:
                        closest = min(closest, abs(u - math.exp(log_a)))
                    if log_a >= 0 or u < math.exp(log_a):
                        s[y0:y0 + Bs, x0:x0 + Bs] = prop
                        acc[r] += 1
    return out, acc, closest


@pytest.mark.parametrize("Bs", [8, 4, 2])
def test_block_round_follows_its_definition(Bs):
    """Two block rounds of a batch (replicas at K = 0.02, 0.15 and 0.45, so
    proposals are both accepted and rejected) against the round computed on the
    host from its definition: the lattices and per-replica accept counts agree
    bit for bit."""
    import torch
    P = _P()
    Lx, Ly = 64, 16
    descs = [dict(Lx=Lx, Ly=Ly, J=1.0, beta=beta, seed=0x5EED0000 + 31 * r, replica=3 + r, init=0)
             for r, beta in enumerate((0.02, 0.15, 0.45))]
    b = P.Batch(descs)
    b.run(30)
    net = P.Net(_params(1.0), block=Bs, max_batch=16, max_seq=256)
    acc = torch.zeros(len(descs), dtype=torch.int64, device="cuda")
    total = np.zeros(len(descs), dtype=np.int64)
    for round_ in (7, 8):
        before = [b.get_spins(r).astype(np.int64) for r in range(len(descs))]
        want, a, closest = _host_block_round(net, before, descs, Bs, round_)
        assert closest > 1e-12, closest
        b.block_round(net, round_, acc)
        torch.cuda.synchronize()
        total += a
        for r in range(len(descs)):
            assert np.array_equal(b.get_spins(r).astype(np.int64), want[r]), (Bs, round_, r)
        assert np.array_equal(acc.cpu().numpy(), total), (acc.cpu().numpy(), total)
    n_blocks = 2 * len(descs) * (Lx // Bs) * (Ly // Bs)
    assert 0 < total.sum() < n_blocks, total


def test_training_entry_points_reject_bad_arguments():
    """Errors of the training entry points come back as ISING_E_INVALID with a
    message, before any work is enqueued: a batch outside [1, max_batch], a
    training set of no rows, a non-positive learning rate, a step count below
    one."""
    import torch
    P = _P()
    rng = np.random.default_rng(5)
    Bs = 4
    x, bnd, kc = _rand_blocks(rng, 40, Bs)
    X, BN, K = _dev(x, torch.int8), _dev(bnd, torch.int8), _dev(kc, torch.float32)
    net = P.Net(_params(1.0), block=Bs, max_batch=32, max_seq=64)
    theta = net.params.copy()
    bad = [lambda: net.train_step_sampled(X, BN, K, 33, 1e-3, 1),
           lambda: net.train_step_sampled(X, BN, K, 0, 1e-3, 1),
           lambda: net.train_step_sampled(X, BN, K, 16, 0.0, 1),
           lambda: net.train_steps_sampled(X, BN, K, 16, 1e-3, 1, 0),
           lambda: net.train_steps_sampled(X[:0], BN[:0], K[:0], 16, 1e-3, 1, 4),
           lambda: net.train_step(X[:33], BN[:33], K[:33], 1e-3)]
    for f in bad:
        with pytest.raises(P.IsingError) as e:
            f()
        assert e.value.code == P.ISING_E_INVALID, e.value
    torch.cuda.synchronize()
    assert np.array_equal(net.params, theta)  # nothing was enqueued
