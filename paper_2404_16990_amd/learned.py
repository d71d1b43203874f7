"""Learned block proposals on a replica batch: training data, training, and
the comparison against plain checkerboard sweeps on effective |m| samples.

Every device step is a library call (see include/ising.h); this module only
schedules them and analyses the recorded traces on the host.
"""
import sys
import time

import numpy as np

from . import Batch, Net, analysis


def collect_blocks(batch: Batch, block: int, per_replica: int, draws: int, sweeps_between: int):
    """Training blocks from the plain sampler: `draws` times, run
    `sweeps_between` sweeps and take `per_replica` blocks of every replica,
    written straight into one preallocated training set."""
    import torch
    per_draw = batch.n * per_replica
    dev = batch.buf.device
    X = torch.empty((draws * per_draw, block * block), dtype=torch.int8, device=dev)
    BN = torch.empty((draws * per_draw, 4 * block), dtype=torch.int8, device=dev)
    K = torch.empty(draws * per_draw, dtype=torch.float32, device=dev)
    for d in range(draws):
        batch.run(sweeps_between)
        s = slice(d * per_draw, (d + 1) * per_draw)
        batch.extract_blocks(block, per_replica, d, out=(X[s], BN[s], K[s]))
    return X, BN, K


def train(net: Net, X, BN, K, steps: int, batch_size: int, lr: float, seed: int = 0, log_every: int = 100):
    """Adam on minibatches the library draws on the device from (X, BN, K);
    returns [(step, loss)] every log_every steps."""
    import torch
    loss = torch.zeros(1, dtype=torch.float32, device=X.device)
    out = []
    marks = sorted(set(list(range(0, steps, log_every)) + [steps - 1]))
    done = 0
    for s in marks:  # steps done .. s in one call, then the loss of step s
        net.train_steps_sampled(X, BN, K, batch_size, lr, seed, s + 1 - done, loss)
        done = s + 1
        out.append((s, float(loss.cpu())))
    return out


def _per_spin(batch: Batch):
    n = np.array([d["Lx"] * d["Ly"] for d in batch.descs], dtype=np.float64)
    j = np.array([d["J"] for d in batch.descs], dtype=np.float64)
    return n, j


def unit_traces(batch: Batch, units: int, unit, progress: int = 0):
    """Run `units` units (callable unit(i) returning device traces (B, M) of
    the unit); returns (|m| trace, e trace) [n_rep, units] and seconds.  With
    progress > 0 the device is drained and a line printed to stderr every
    `progress` units (a long run then reports as it goes)."""
    import torch
    n, j = _per_spin(batch)
    bonds, mags = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(units):
        b, m = unit(i)
        bonds.append(b)
        mags.append(m)
        if progress and (i + 1) % progress == 0 and i + 1 < units:
            torch.cuda.synchronize()
            print(f"learned units: {i + 1} of {units}, {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    B = np.concatenate([t.cpu().numpy() for t in bonds], axis=1).astype(np.float64)
    M = np.concatenate([t.cpu().numpy() for t in mags], axis=1).astype(np.float64)
    return np.abs(M) / n[:, None], -j[:, None] * B / n[:, None], dt


def plain_trace(batch: Batch, sweeps: int, record_every: int):
    """One run of `sweeps` plain sweeps recording (B, M) every `record_every`;
    returns (|m| trace, e trace) [n_rep, sweeps/record_every] and seconds of
    device time."""
    import torch
    n, j = _per_spin(batch)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(batch.stream)
    bond, mag = batch.run(sweeps, record_every)
    e1.record(batch.stream)
    torch.cuda.synchronize()
    B = bond.cpu().numpy().astype(np.float64)
    M = mag.cpu().numpy().astype(np.float64)
    return np.abs(M) / n[:, None], -j[:, None] * B / n[:, None], e0.elapsed_time(e1) / 1e3


def learned_units(batch: Batch, net: Net, first_round: int, accepts=None):
    """One unit = one block round (both block colours) then one checkerboard
    sweep; returns the sweep's (B, M) trace."""
    def unit(i):
        batch.block_round(net, first_round + i, accepts)
        return batch.run(1, 1)
    return unit


def summarise(trace, seconds, units_per_trace_point, replicas):
    """tau_int (in trace points) of |m|, Sokal's windowed estimate averaged over
    the independent replicas `replicas` (same temperature), with the standard
    error of that mean, and the effective samples per second it gives (per
    replica, whole-batch time)."""
    taus = np.array([analysis.tau_int(trace[r])[0] for r in replicas])
    tau = float(taus.mean())
    points_per_s = trace.shape[1] / seconds
    return {"tau_int_points": tau,
            "tau_int_points_error": float(taus.std(ddof=1) / np.sqrt(len(taus))) if len(taus) > 1 else None,
            "tau_int_points_each": [round(float(t), 2) for t in taus], "points": int(trace.shape[1]),
            "units_per_point": units_per_trace_point, "seconds": seconds,
            "effective_samples_per_s": analysis.effective_rate(points_per_s, tau),
            "run_over_tau": trace.shape[1] / tau}


def replica_agreement(tr_a, tr_b, groups):
    """Per group of independent replicas at one temperature, z of the
    difference of the two samplers' means of an observable: each replica's
    run mean is one sample, and the error of a sampler's group mean is the
    spread of those samples over sqrt(n) (no autocorrelation time enters).
    For n = 8 replicas a side the z's follow Student's t with about 14
    degrees of freedom: |z| < 2 for 93.5 % of the groups."""
    zs = []
    for g in groups:
        ma, mb = tr_a[g].mean(axis=1), tr_b[g].mean(axis=1)
        se = np.sqrt(ma.var(ddof=1) / len(g) + mb.var(ddof=1) / len(g))
        zs.append((ma.mean() - mb.mean()) / se if se > 0 else 0.0)
    return np.array(zs)


def agreement(tr_a, tr_b, n_bins=0):
    """Per replica z of the mean of two traces: errors from Sokal's windowed
    tau_int (n_bins = 0) or from batch means over n_bins bins."""
    zs = []
    for r in range(tr_a.shape[0]):
        if n_bins:
            ma, ea = analysis.batch_means_error(tr_a[r], n_bins)
            mb, eb = analysis.batch_means_error(tr_b[r], n_bins)
        else:
            ta, _ = analysis.tau_int(tr_a[r])
            tb, _ = analysis.tau_int(tr_b[r])
            ma, ea = analysis.mean_and_error(tr_a[r], ta)
            mb, eb = analysis.mean_and_error(tr_b[r], tb)
        zs.append((ma - mb) / np.sqrt(ea * ea + eb * eb) if ea + eb > 0 else 0.0)
    return np.array(zs)


def agreement_summary(z):
    """Fraction of |z| < 2 (0.954 for correct Gaussian errors), max |z| and
    chi^2 per degree of freedom, mean(z^2) (1 for correct errors)."""
    z = np.asarray(z, dtype=np.float64)
    return {"within_2sigma": float(np.mean(np.abs(z) < 2)), "max_abs_z": float(np.max(np.abs(z))),
            "chi2_per_dof": float(np.mean(z * z))}
