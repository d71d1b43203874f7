"""Float64 numpy reference of the block-proposal network (test infrastructure).

The network proposes a joint update of one Bs x Bs block of spins given the
block's boundary spins and beta, one site at a time in raster order
(k = i*Bs + j, i = row, j = column), so that the proposal probability q is a
product of tractable conditionals; Metropolis-Hastings with that q keeps the
Boltzmann distribution of section 1 of the paper exact.  Nothing here is
called by the GPU library; tests compare the library's kernels with it.

Architecture (parameters in one flat float vector, order below; C channels):
  layer 1, taps A = {(-1,-1), (-1,0), (-1,1), (0,-1)} over the spin field:
    pre1[p,c] = sum_t x[p+t] W1[t,c] + sum_f bnd[p,f] U1[f,c] + beta v1[c] + b1[c]
  layers 2..4, taps B = A + {(0,0)}:
    pre_l[p,c] = sum_t sum_c' h_{l-1}[p+t,c'] W_l[t,c',c] + b_l[c]
  h_l = tanh(pre_l); logit[p] = sum_c h4[p,c] wo[c] + bo
  P(x_p = +1 | x_<p, boundary, beta) = sigmoid(logit[p])
Outside the block the spin field and activations are zero.  bnd[p] holds the
four boundary spins next to site p (up, down, left, right), 0 where the site
is not on that edge.  Tap offsets are (row, column).
"""
import math

import numpy as np

TAPS_A = [(-1, -1), (-1, 0), (-1, 1), (0, -1)]
TAPS_B = TAPS_A + [(0, 0)]


def param_count(C):
    return 4 * C + 4 * C + C + C + 3 * (5 * C * C + C) + C + 1


def unpack(theta, C):
    """Split the flat parameter vector into named arrays (views)."""
    theta = np.asarray(theta)
    o = 0

    def take(shape):
        nonlocal o
        n = int(np.prod(shape))
        a = theta[o:o + n].reshape(shape)
        o += n
        return a

    P = {"W1": take((4, C)), "U1": take((4, C)), "v1": take((C,)), "b1": take((C,))}
    for l in (2, 3, 4):
        P[f"W{l}"] = take((5, C, C))
        P[f"b{l}"] = take((C,))
    P["wo"] = take((C,))
    P["bo"] = take((1,))
    assert o == len(theta)
    return P


def boundary_features(bnd, Bs):
    """bnd: (..., 4*Bs) boundary spins [top row (j), bottom row (j), left column
    (i), right column (i)] -> per-site features (..., Bs, Bs, 4)."""
    bnd = np.asarray(bnd, dtype=np.float64)
    lead = bnd.shape[:-1]
    f = np.zeros(lead + (Bs, Bs, 4))
    f[..., 0, :, 0] = bnd[..., 0:Bs]
    f[..., Bs - 1, :, 1] = bnd[..., Bs:2 * Bs]
    f[..., :, 0, 2] = bnd[..., 2 * Bs:3 * Bs]
    f[..., :, Bs - 1, 3] = bnd[..., 3 * Bs:4 * Bs]
    return f


def _shift(a, di, dj):
    """out[..., i, j, :] = a[..., i+di, j+dj, :] with zeros outside (a has a trailing channel axis)."""
    Bs = a.shape[-2]
    out = np.zeros_like(a)
    i0, i1 = max(0, -di), min(Bs, Bs - di)
    j0, j1 = max(0, -dj), min(Bs, Bs - dj)
    out[..., i0:i1, j0:j1, :] = a[..., i0 + di:i1 + di, j0 + dj:j1 + dj, :]
    return out


def _unshift(g, di, dj):
    """Adjoint of _shift: scatter g[..., i, j] back to position (i+di, j+dj)."""
    Bs = g.shape[-2]
    out = np.zeros_like(g)
    i0, i1 = max(0, -di), min(Bs, Bs - di)
    j0, j1 = max(0, -dj), min(Bs, Bs - dj)
    out[..., i0 + di:i1 + di, j0 + dj:j1 + dj, :] += g[..., i0:i1, j0:j1, :]
    return out


def bf16_round(a):
    """Round float64 values to the nearest bfloat16 (ties to even), via float32."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(theta, C, x, bnd, beta, bf16=False):
    """Teacher-forced logits of a batch of blocks.

    x: (N, Bs, Bs) spins +-1; bnd: (N, 4*Bs) boundary spins; beta: (N,).
    With bf16=True the weights of layers 2..4 and their inputs h1..h3 are
    rounded to bfloat16 first (the precision of the matrix-core layers);
    everything else stays float64.
    Returns (logits (N, Bs, Bs), cache for backward).
    """
    P = unpack(np.asarray(theta, dtype=np.float64), C)
    if bf16:
        P = dict(P)
        for l in (2, 3, 4):
            P[f"W{l}"] = bf16_round(P[f"W{l}"])
    x = np.asarray(x, dtype=np.float64)
    N, Bs, _ = x.shape
    beta = np.asarray(beta, dtype=np.float64).reshape(N, 1, 1, 1)
    feats = boundary_features(bnd, Bs)
    xs = x[..., None]
    pre = np.zeros((N, Bs, Bs, C))
    for t, (di, dj) in enumerate(TAPS_A):
        pre += _shift(xs, di, dj) * P["W1"][t]
    pre += feats @ P["U1"] + beta * P["v1"] + P["b1"]
    hs = [np.tanh(pre)]
    for l in (2, 3, 4):
        h = bf16_round(hs[-1]) if bf16 else hs[-1]
        pre = np.zeros((N, Bs, Bs, C))
        for t, (di, dj) in enumerate(TAPS_B):
            pre += _shift(h, di, dj) @ P[f"W{l}"][t]
        pre += P[f"b{l}"]
        hs.append(np.tanh(pre))
    logits = hs[-1] @ P["wo"] + P["bo"][0]
    return logits, {"x": xs, "feats": feats, "beta": beta, "hs": hs, "P": P}


def nll(logits, x):
    """Mean over sites of -log P(x | logit) = softplus(-x * logit)."""
    z = -np.asarray(x, dtype=np.float64) * logits
    return float(np.mean(np.logaddexp(0.0, z)))


def loss_and_grad(theta, C, x, bnd, beta, bf16=False):
    """Mean per-site negative log-likelihood and its gradient (flat, float64).

    With bf16=True the gradient is evaluated at the rounding points of the
    matrix-core layers: the forward is forward(..., bf16=True), and in the
    backward the gradient of each layer-2..4 pre-activation is rounded to
    bfloat16 before it enters the two products of that layer (its weight
    gradient against the bfloat16 inputs, and the gradient passed to the
    layer below through the bfloat16 weights).  Bias and layer-1 gradients
    use the unrounded values; the loss is always the exact one.
    """
    logits, cache = forward(theta, C, x, bnd, beta, bf16=bf16)
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    loss = nll(logits, x)
    # d/dlogit softplus(-x l) = -x * sigmoid(-x l)
    dlogit = -x / (1.0 + np.exp(x * logits)) / n
    P = cache["P"]
    hs = cache["hs"]
    G = {k: np.zeros_like(v) for k, v in P.items()}
    G["wo"] = np.einsum("nijc,nij->c", hs[-1], dlogit)
    G["bo"] = np.array([dlogit.sum()])
    dh = dlogit[..., None] * P["wo"]
    for l in (4, 3, 2):
        dpre = dh * (1.0 - hs[l - 1] ** 2)
        G[f"b{l}"] = dpre.sum(axis=(0, 1, 2))
        hin = bf16_round(hs[l - 2]) if bf16 else hs[l - 2]
        if bf16:
            dpre = bf16_round(dpre)
        dh = np.zeros_like(hin)
        for t, (di, dj) in enumerate(TAPS_B):
            G[f"W{l}"][t] = np.einsum("nijc,nijd->cd", _shift(hin, di, dj), dpre)
            dh += _unshift(dpre @ P[f"W{l}"][t].T, di, dj)
    dpre = dh * (1.0 - hs[0] ** 2)
    for t, (di, dj) in enumerate(TAPS_A):
        G["W1"][t] = np.einsum("nij,nijc->c", _shift(cache["x"], di, dj)[..., 0], dpre)
    G["U1"] = np.einsum("nijf,nijc->fc", cache["feats"], dpre)
    G["v1"] = np.einsum("n,nijc->c", cache["beta"][:, 0, 0, 0], dpre)
    G["b1"] = dpre.sum(axis=(0, 1, 2))
    flat = np.concatenate([G[k].ravel() for k in P.keys()])
    return loss, flat


def threshold(logit):
    """Proposal threshold: P(+1) = thr / 2^32, thr = clamp(floor(sigmoid(logit) 2^32), 1, 2^32-1)."""
    p = 1.0 / (1.0 + math.exp(-float(logit)))
    return int(min(max(math.floor(p * 4294967296.0), 1), 4294967295))


def log_q(theta, C, x, bnd, beta, bf16=False):
    """log q(x | boundary, beta) of one block from thresholds (float64)."""
    logits, _ = forward(theta, C, np.asarray(x)[None], np.asarray(bnd)[None], np.asarray([beta]), bf16=bf16)
    Bs = logits.shape[1]
    s = 0.0
    for i in range(Bs):
        for j in range(Bs):
            thr = threshold(logits[0, i, j])
            s += math.log(thr if x[i][j] > 0 else 4294967296 - thr) - 32 * math.log(2.0)
    return s


def sample(theta, C, bnd, beta, uniforms):
    """Draw one block site by site: x_k = +1 iff uniforms[k] < thr_k (uint32 uniforms)."""
    Bs = int(round(math.sqrt(len(uniforms))))
    x = np.zeros((Bs, Bs))
    for k in range(Bs * Bs):
        i, j = divmod(k, Bs)
        logits, _ = forward(theta, C, x[None], np.asarray(bnd)[None], np.asarray([beta]))
        x[i, j] = 1.0 if uniforms[k] < threshold(logits[0, i, j]) else -1.0
    return x


def adam_step(theta, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One step of Adam (Kingma and Ba, 2015, Algorithm 1) in float64.

    t is the 1-based step number; m, v the first and second moment estimates
    before the step (zeros before the first).  Returns (theta', m', v'):
      m' = b1 m + (1 - b1) g,   v' = b2 v + (1 - b2) g^2,
      theta' = theta - lr (m' / (1 - b1^t)) / (sqrt(v' / (1 - b2^t)) + eps).
    """
    g = np.asarray(grad, dtype=np.float64)
    m2 = b1 * np.asarray(m, dtype=np.float64) + (1.0 - b1) * g
    v2 = b2 * np.asarray(v, dtype=np.float64) + (1.0 - b2) * g * g
    mhat = m2 / (1.0 - b1 ** t)
    vhat = v2 / (1.0 - b2 ** t)
    return np.asarray(theta, dtype=np.float64) - lr * mhat / (np.sqrt(vhat) + eps), m2, v2


def thresholds(logits):
    """Vectorised threshold() over an array of logits (uint64 values)."""
    p = 1.0 / (1.0 + np.exp(-np.asarray(logits, dtype=np.float64)))
    return np.clip(np.floor(p * 4294967296.0), 1, 4294967295).astype(np.uint64)


def sample_batch(theta, C, bnd, beta, uniforms, bf16=False):
    """sample() for N blocks at once: uniforms (N, Bs*Bs) uint32; site k of
    every block is drawn from the logits of the blocks drawn so far.
    Returns (x (N, Bs, Bs) of +-1, thresholds (N, Bs*Bs) used at each site)."""
    u = np.asarray(uniforms, dtype=np.uint64)
    N, BB = u.shape
    Bs = int(round(math.sqrt(BB)))
    x = np.zeros((N, Bs, Bs))
    thr = np.zeros((N, BB), dtype=np.uint64)
    beta = np.asarray(beta, dtype=np.float64)
    for k in range(BB):
        i, j = divmod(k, Bs)
        logits, _ = forward(theta, C, x, bnd, beta, bf16=bf16)
        thr[:, k] = thresholds(logits[:, i, j])
        x[:, i, j] = np.where(u[:, k] < thr[:, k], 1.0, -1.0)
    return x, thr


def log_q_batch(theta, C, x, bnd, beta, bf16=False):
    """log_q() for N blocks at once: x (N, Bs, Bs) of +-1.  Returns (log q (N,),
    per-site logits (N, Bs, Bs))."""
    x = np.asarray(x, dtype=np.float64)
    logits, _ = forward(theta, C, x, bnd, beta, bf16=bf16)
    thr = thresholds(logits).astype(np.float64)
    chosen = np.where(x > 0, thr, 4294967296.0 - thr)
    return (np.log(chosen) - 32 * math.log(2.0)).sum(axis=(1, 2)), logits
