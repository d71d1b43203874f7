"""The paper's validation campaign on the batched path (section 3.1): <|m|>(T)
for many temperatures and several lattice sizes, each from a completely random
start, the non-equilibrated beginning of every |m| trace discarded by the
automatic detection of analysis.equilibration, compared with the exact
spontaneous magnetisation of the infinite lattice, [1 - sinh(2J/T)^-4]^(1/8),
below T_c and with the finite lattice's <|m|> (finite_size_m) above.

Usage: python -m paper_2404_16990_amd.validation --sizes 1024 2048 \
           --sweeps 200000 --every 1000 --rng bitsliced --out campaign.json
(--cluster-burnin N first equilibrates the random starts with N Swendsen-Wang
steps, which removes the domain coarsening that single-spin sweeps from a
random start need below T_c.)
Every device step is a library call; this module only schedules runs and
analyses the recorded traces on the host.
"""
import argparse
import json
import math
import sys
import time

import numpy as np

from . import Batch, analysis

T_C = 2.0 / math.log(1.0 + math.sqrt(2.0))


# Amplitude of the high-temperature susceptibility of the square lattice,
# chi ~ C (1 - T_c/T)^(-7/4) as T -> T_c from above (Wu, McCoy, Tracy and
# Barouch, 1976).
CHI_AMPLITUDE = 0.9625817322


def spontaneous_m(T, J=1.0):
    """Exact |m| of the infinite lattice (Yang's result as quoted in section 3.1)."""
    if T >= T_C * J:
        return 0.0
    return (1.0 - math.sinh(2.0 * J / T) ** -4) ** 0.125


def finite_size_m(T, L, J=1.0):
    """<|m|> of an L x L torus above T_c to leading order, for L much larger
    than the correlation length: m is then Gaussian with variance chi / N, so
    <|m|> = (2 chi / (pi N))^(1/2), with chi from its leading critical form.
    The infinite lattice's 0 is not what a finite lattice shows just above T_c
    (0.022 at T = 2.32 on 1024^2)."""
    t = 1.0 - T_C * J / T
    chi = CHI_AMPLITUDE * t ** -1.75
    return math.sqrt(2.0 * chi / (math.pi * L * L))


def expected_m(T, L, J=1.0):
    """The comparison value: Yang's m below T_c, the finite-size <|m|> above."""
    return spontaneous_m(T, J) if T < T_C * J else finite_size_m(T, L, J)


def run_size(L, temps, sweeps, every, rng, seed0=16990, chunks=10, log=print, cluster_burnin=0,
             keep_traces=False):
    """One size of the campaign.  With cluster_burnin > 0 the random starts
    are first equilibrated by that many Swendsen-Wang steps (same batch, same
    step counter); the measured trace is always Metropolis sweeps.  With
    keep_traces the result also holds the recorded magnetisations M (int64,
    replicas x sweeps // every) under "mag"."""
    import torch
    descs = [dict(Lx=L, Ly=L, J=1.0, beta=1.0 / T, seed=seed0 + i, replica=i, init=0, rng=rng)
             for i, T in enumerate(temps)]
    b = Batch(descs)
    burnin_s = 0.0
    if cluster_burnin > 0:
        t0 = time.perf_counter()
        b.cluster(cluster_burnin, "sw")
        torch.cuda.synchronize()
        burnin_s = time.perf_counter() - t0
        b.ws = None
        torch.cuda.empty_cache()
        log(f"L={L}: {cluster_burnin} Swendsen-Wang steps, {burnin_s:.1f} s")
    b.autotune(trial_sweeps=5)
    n = float(L * L)
    traces = []
    per = sweeps // chunks
    t0 = time.perf_counter()
    for c in range(chunks):
        _, mag = b.run(per, every)
        traces.append(mag.cpu().numpy())
        log(f"L={L}: {(c + 1) * per} of {sweeps} sweeps, {time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    seconds = time.perf_counter() - t0
    b.close()
    mag = np.concatenate(traces, axis=1)
    rows = analyse(mag, temps, L, every)
    out = {"L": L, "sweeps": sweeps, "every": every, "seconds": seconds, "cluster_burnin": cluster_burnin,
           "cluster_burnin_s": burnin_s, "flips_per_s": len(temps) * n * sweeps / seconds, "rows": rows}
    if keep_traces:
        out["mag"] = mag
    return out


def analyse(mag, temps, L, every):
    """Per temperature: the equilibration point of the |m| trace (Chodera's
    automatic detection), <|m|> after it with its tau-corrected error, and
    the comparison values."""
    m = np.abs(np.asarray(mag, dtype=np.float64)) / float(L * L)
    rows = []
    for i, T in enumerate(temps):
        t_eq, g, n_eff = analysis.equilibration(m[i])
        x = m[i, t_eq:]
        tau, _ = analysis.tau_int(x)
        mean, err = analysis.mean_and_error(x, tau)
        rows.append({"T": round(float(T), 6), "m": mean, "err": err, "exact": spontaneous_m(T),
                     "expected": expected_m(float(T), L),
                     "t_eq_sweeps": int(t_eq * every), "n_eff": float(n_eff)})
    return rows


def summarise(res, band=0.05):
    """Agreement away from T_c (|T - T_c| > band): |<|m|> - expected| < 0.01
    (Yang's m below T_c, the finite-size <|m|> above), and the replicas that
    miss it (stripe states frozen at low T, slow ones near T_c)."""
    ok, miss = 0, []
    for r in res["rows"]:
        if abs(r["T"] - T_C) <= band:
            continue
        want = expected_m(r["T"], res["L"])
        if abs(r["m"] - want) < 0.01:
            ok += 1
        else:
            miss.append((r["T"], round(r["m"], 4), round(want, 4)))
    return {"L": res["L"], "agree": ok, "checked": ok + len(miss), "misses": miss}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", type=int, nargs="+", default=[1024])
    ap.add_argument("--t-min", type=float, default=0.385)
    ap.add_argument("--t-max", type=float, default=4.145)
    ap.add_argument("--dt", type=float, default=0.005)
    ap.add_argument("--sweeps", type=int, default=200000)
    ap.add_argument("--every", type=int, default=1000)
    ap.add_argument("--rng", default="bitsliced", choices=["site", "bitsliced"])
    ap.add_argument("--cluster-burnin", type=int, default=0,
                    help="Swendsen-Wang steps before the Metropolis sweeps (0: none, as in the paper)")
    ap.add_argument("--out", default="", help="JSON file for every row of every size")
    ap.add_argument("--summary", default="",
                    help="JSON file for the agreement summary of each size, its timing and the command line")
    args = ap.parse_args()
    temps = np.round(np.arange(args.t_min, args.t_max + 0.5 * args.dt, args.dt), 6)
    rng = 1 if args.rng == "bitsliced" else 0
    results = []
    for L in args.sizes:
        res = run_size(L, temps, args.sweeps, args.every, rng, log=lambda s: print(s, flush=True),
                       cluster_burnin=args.cluster_burnin)
        results.append(res)
        print(json.dumps(summarise(res)), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump({"rng": args.rng, "results": results}, f)
    if args.summary:
        sizes = []
        for res in results:
            keep = ("L", "sweeps", "every", "seconds", "cluster_burnin", "cluster_burnin_s", "flips_per_s")
            e = {k: res[k] for k in keep}
            e["summary"] = summarise(res)
            e["rows_every_0.25"] = [r for r in res["rows"] if abs(round(r["T"] / 0.25) * 0.25 - r["T"]) < 1e-9]
            sizes.append(e)
        with open(args.summary, "w") as f:
            json.dump({"command": "python -m paper_2404_16990_amd.validation " + " ".join(sys.argv[1:]),
                       "rng": args.rng, "temperatures": len(temps), "sizes": sizes}, f, indent=1)


if __name__ == "__main__":
    main()
