"""Throughput benchmark: aggregate flip attempts per second on one MI355X.

Workload (default): 256 replicas of 1024x1024 periodic lattices, J = 1,
T_r = 1.5 + 2 r / 255, seed 16990 + r, random start; (B, M) recorded every 100
sweeps.  One step = 100 checkerboard sweeps of every replica (each sweep
updates both colours), so the default 100 timed steps are the full 10^4-sweep
run.  The lattices are resident in HBM before timing starts.

Prints ONE JSON line with the metric, the roofline of the dominant kernel, and
the CPU oracle's rate on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published figures used for the roofline (see the design notes)
CUS, LANES_PER_CU, CLOCK_HZ = 256, 64, 2.4e9
# lane-cycles of the minimal instruction sequence for one flip attempt: a
# quarter of a Philox4x32-10 call (5 full 32x32->64 products at quarter rate
# = 20, 5 three-input XORs = 5) plus one threshold compare
LANE_CYCLES_PER_FLIP = 26.0
HBM_BYTES_PER_S = 8.0e12


def alu_peak_flips():
    return CUS * LANES_PER_CU * CLOCK_HZ / LANE_CYCLES_PER_FLIP


def host_threads():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_baseline(work, sweeps):
    """Time the CPU oracle on every replica of the workload for `sweeps` sweeps."""
    import oracle
    descs = [oracle.desc(r.Lx, r.Ly, r.J, r.beta, r.seed, r.replica, r.init) for r in work.replicas]
    states = [oracle.init_state(d) for d in descs]
    threads = host_threads()
    t0 = time.perf_counter()
    oracle.run_batch(descs, states, sweeps, threads=threads)
    dt = time.perf_counter() - t0
    flips = work.spins * sweeps
    return {"value": flips / dt, "unit": "flip attempts/s", "cores": threads, "kind": "oracle",
            "sample": f"all {len(work.replicas)} replicas x {sweeps} sweeps (of {work.sweeps}), "
                      f"{dt:.1f} s on {threads} host threads"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--sweeps-per-step", type=int, default=100)
    ap.add_argument("--workload", default="batch_256x1024")
    ap.add_argument("--cpu-sweeps", type=int, default=40)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--schedule", default="", help="JSON dict overriding the execution schedule")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(replicas would shard across GPUs with no communication).", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2404_16990_amd as P
    import workloads

    work = workloads.ALL[args.workload]()
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    descs = [dict(Lx=r.Lx, Ly=r.Ly, J=r.J, beta=r.beta, seed=r.seed, replica=r.replica, init=r.init)
             for r in work.replicas]
    batch = P.Batch(descs, stream=stream)
    if args.schedule:
        batch.set_schedule(**json.loads(args.schedule))
    sched = batch.schedule
    n_res, n_str = batch.mode_counts()
    spw = args.sweeps_per_step
    rec_every = min(work.record_every, spw)

    def step():
        return batch.run(spw, rec_every)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    traces = []
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    ev[0].record(stream)
    for k in range(args.steps):
        traces.append(step())
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    step_ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]
    total_s = sum(step_ms) / 1e3
    flips = work.spins * spw * args.steps
    value = flips / total_s

    # dominant kernel: each step is spw / sweeps_per_launch graph launches of the
    # sweep kernel (plus a one-thread-per-replica counter kernel)
    launches_per_step = max(1, spw // sched["sweeps_per_launch"])
    launch_s = (total_s / args.steps) / launches_per_step
    flips_per_launch = work.spins * min(spw, sched["sweeps_per_launch"])
    achieved = flips_per_launch / launch_s
    peak = alu_peak_flips()
    kernel = "k_sweep_resident" if n_str == 0 else ("k_sweep_stream" if n_res == 0 else "mixed")
    roofline = {"bound": "alu", "kernel": kernel, "achieved": achieved / 1e9, "peak": peak / 1e9,
                "unit": "Gflip/s", "frac": achieved / peak, "traffic": None,
                "per_unit": f"{LANE_CYCLES_PER_FLIP:g} VALU lane-cycles per flip attempt",
                "launch_ms": launch_s * 1e3}
    # sanity: the last trace is finite and physical
    b_last = traces[-1][0][:, -1].cpu()
    assert int(b_last.abs().max()) <= 2 * max(r.spins for r in work.replicas)

    out = {
        "metric": "aggregate flip attempts/s on 1 MI355X",
        "value": value,
        "unit": "flip attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_s * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32 (1 bit/spin, integer Philox thresholds)",
        "data": "synthetic",
        "config": {"workload": work.name, "replicas": len(work.replicas), "spins": work.spins,
                   "sweeps_per_step": spw, "record_every": rec_every, "schedule": sched,
                   "resident_replicas": n_res, "streamed_replicas": n_str,
                   "wall_s": wall},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(work, args.cpu_sweeps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
