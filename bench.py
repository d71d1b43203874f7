"""Throughput benchmark: aggregate flip attempts per second on one MI355X.

Headline workload (default): the uneven batch of 512 periodic square
lattices, sides 2^k with k uniform on {7..13} (128^2 .. 8192^2, 6.9e9 spins in
all) and T uniform on [2.0, 2.6), both from numpy PCG64(16990); J = 1,
seed 16990 + r, random start; (B, M) recorded every 100 sweeps.  One step = 100
checkerboard sweeps of every replica (each sweep updates both colours), so the
default 20 timed steps are the workload's full 2000-sweep run.  The lattices
are resident in HBM before timing starts; the schedule comes from the
library's autotuner.

Prints ONE JSON line with the metric, the roofline of the dominant kernel, the
CPU oracle's rate on a bounded sample of the same workload, the other plain
configurations (256 x 1024^2; 754 x 512x528 + 16384x12288) timed the same way,
and the learned-proposal comparison at T_c (effective independent |m| samples
per second against plain sweeps).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs at 2.4 GHz.  Each CU has four SIMDs of 16 lanes; a wave64
# VALU instruction occupies its SIMD for 4 clocks, so plain (non-packed)
# 32-bit integer instructions issue at 64 lane-operations per CU per clock
# (the published fp64 vector rate, 78.6 TFLOP/s, is the same 64 FMA lanes per
# CU per clock; the fp32 figure of 157.3 TFLOP/s counts two packed fp32
# operations per lane, which integer work cannot use).
CUS, LANE_OPS_PER_CU_CLK, CLOCK_HZ = 256, 64, 2.4e9
# VALU instructions of the algorithmic work of one flip attempt: a quarter of
# one Philox4x32-10 call (20 32x32->64 products and 20 three-input XORs per
# call, i.e. 5 + 5), the acceptance (threshold select, compare, bit insert: 3)
# and one instruction of neighbour words, classification and flip amortised
# over the 32 sites of a word.
OPS_PER_FLIP = 5 + 5 + 3 + 1
HBM_BYTES_PER_S = 8.0e12


def lane_ops_peak():
    return CUS * LANE_OPS_PER_CU_CLK * CLOCK_HZ


def alu_peak_flips():
    return lane_ops_peak() / OPS_PER_FLIP


SWEEP_SOURCES = ("paper_2404_16990_amd/csrc/kernels.hip", "paper_2404_16990_amd/csrc/device.hpp",
                 "paper_2404_16990_amd/csrc/launch.hpp")
CLUSTER_SOURCES = ("paper_2404_16990_amd/csrc/cluster.hip", "paper_2404_16990_amd/csrc/cluster.hpp",
                   "paper_2404_16990_amd/csrc/device.hpp")


def kernel_source_digest(sources=SWEEP_SOURCES):
    import hashlib
    h = hashlib.sha256()
    for rel in sources:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


TRAFFIC_FILES = {"k_sweep_stream": "traffic_k_sweep_stream_uneven512.json",
                 "k_sweep_resident": "traffic_k_sweep_resident_batch256x1024.json"}


def measured_traffic(kernel, workload_name, sweeps_per_launch):
    """HBM bytes per launch from the committed counter summary of `kernel`, or
    None when the summary is for another workload or launch length or the
    kernel sources changed since the counters were taken."""
    name = TRAFFIC_FILES.get(kernel)
    if name is None:
        return None, None
    try:
        with open(os.path.join(ROOT, "profiles", name)) as f:
            d = json.load(f)
    except OSError:
        return None, None
    if d.get("kernel_source_sha256") != kernel_source_digest():
        return None, None
    if not d["kernel"].startswith(kernel) or not d["workload"].startswith(workload_name):
        return None, None
    e = d["by_sweeps_per_launch"].get(str(sweeps_per_launch))
    if e is None:
        return None, None
    return e["traffic_bytes_per_launch"], e.get("algorithmic_bytes_per_launch", d["algorithmic_bytes_per_launch"])


def measured_cluster_traffic(workload_name):
    """HBM bytes of one Swendsen-Wang step from the committed counter summary,
    or None when it is for another workload or the cluster sources changed."""
    try:
        with open(os.path.join(ROOT, "profiles", "traffic_cluster_sw_batch256x1024.json")) as f:
            d = json.load(f)
    except OSError:
        return None
    if d.get("kernel_source_sha256") != kernel_source_digest(CLUSTER_SOURCES):
        return None
    if not d["workload"].startswith(workload_name):
        return None
    return d["traffic_bytes_per_step"]


def host_threads():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_baseline(work, sweeps, rng=0):
    """Time the CPU oracle on every replica of the workload for `sweeps` sweeps
    under the measured path's random-number contract."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    descs = [oracle.desc(r.Lx, r.Ly, r.J, r.beta, r.seed, r.replica, r.init, rng=rng) for r in work.replicas]
    threads = host_threads()
    # initial states (untimed) on all host threads: the library calls release the GIL
    with ThreadPoolExecutor(threads) as pool:
        states = list(pool.map(oracle.init_state, descs))
    t0 = time.perf_counter()
    oracle.run_batch(descs, states, sweeps, threads=threads)
    dt = time.perf_counter() - t0
    flips = work.spins * sweeps
    return {"value": flips / dt, "unit": "flip attempts/s", "cores": threads, "kind": "oracle",
            "sample": f"all {len(work.replicas)} replicas x {sweeps} sweeps (of {work.sweeps}), "
                      f"{dt:.1f} s on {threads} host threads"}


# Schedule the autotuner starts from (its incumbent) per workload.  The
# uneven batch starts all-streamed: a mixed placement (lattices up to 1024^2
# resident in LDS beside the streamed ones) must then be 2 % faster to be
# chosen, and when it is not, every launch of the timed region is one
# streaming kernel, whose mean duration the events and the kernel trace give
# directly.
TUNE_START = {"uneven-512-L128..8192": {"resident_max_bytes": 0}}


def run_path(work, rng, args, stream, schedule=None):
    """Create the batch under random-number contract `rng`, pick its schedule
    (given, or from the autotuner), warm up, and time args.steps steps.
    Returns the measurement and the batch."""
    import torch

    import paper_2404_16990_amd as P

    descs = [dict(Lx=r.Lx, Ly=r.Ly, J=r.J, beta=r.beta, seed=r.seed, replica=r.replica, init=r.init, rng=rng)
             for r in work.replicas]
    batch = P.Batch(descs, stream=stream)
    tuned = None
    if schedule:
        batch.set_schedule(**schedule)
    elif not args.no_autotune:
        if work.name in TUNE_START:
            batch.set_schedule(**TUNE_START[work.name])
        t0 = time.perf_counter()
        _, n_tried = batch.autotune(trial_sweeps=args.tune_sweeps)
        tuned = {"candidates": n_tried, "seconds": time.perf_counter() - t0}
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
    # sanity: the last trace is finite and physical
    b_last = traces[-1][0][:, -1].cpu()
    assert int(b_last.abs().max()) <= 2 * max(r.spins for r in work.replicas)

    # dominant kernel: all-resident batches launch one k_sweep_resident per
    # sweeps_per_launch sweeps; all-streaming batches one k_sweep_stream per
    # colour per sweep and per word-width list present (the 64-bit list holds
    # every replica with Lx % 128 == 0, the 32-bit list the rest).  Launches on
    # the stream are back to back, so the mean launch duration is the timed
    # region over the number of launches (it includes the one-thread-per-replica
    # counter kernel after each chunk).
    S = sched["sweeps_per_launch"]
    n_lists = 1
    if sched["word_bits"] == 64 and any(r.Lx % 128 for r in work.replicas) and \
            any(r.Lx % 128 == 0 for r in work.replicas):
        n_lists = 2
    if n_str == 0:
        kernel, launches, flips_per_launch = "k_sweep_resident", args.steps * -(-spw // S) * n_lists, \
            work.spins * min(spw, S) / n_lists
    elif n_res == 0:
        kernel, launches, flips_per_launch = "k_sweep_stream", args.steps * spw * 2 * n_lists, \
            work.spins * 0.5 / n_lists
    else:
        # mixed: per chunk of S sweeps, 2 S streaming launches back to back on
        # the stream, the resident replicas' one launch beside them on a second
        # stream; the chunk (both kernels' work) is the unit timed
        kernel, launches, flips_per_launch = \
            f"k_sweep_stream ({2 * min(spw, S)} launches per chunk) + k_sweep_resident (concurrent)", \
            args.steps * -(-spw // S), work.spins * min(spw, S)
    launch_s = total_s / launches
    achieved = flips_per_launch / launch_s
    return {"value": flips / total_s, "ms_per_step": total_s * 1e3 / args.steps, "schedule": sched,
            "resident_replicas": n_res, "streamed_replicas": n_str, "autotune": tuned, "wall_s": wall,
            "kernel": kernel, "launches": launches, "launch_s": launch_s, "achieved": achieved,
            "flips_per_launch": flips_per_launch, "rec_every": rec_every}, batch


RNG_NAMES = {"site": 0, "bitsliced": 1}

# Work of one Swendsen-Wang step per site that the library's random-number
# contract fixes: half a Philox4x32-10 call for the two bonds a site owns (40
# VALU instructions per call) and at most 1/128 of a call for the flip bits
# (one call serves 128 consecutive root indices); the HBM traffic of the
# step's data layout is a 32-bit label written and read back plus the spin
# bits read twice and written once (1 bit per site each, 1.5x for the
# neighbour rows of the bond pass).  The traffic bound is the lower one.
PHILOX_OPS = 20 + 20
SW_OPS_PER_SITE = (0.5 + 1.0 / 128.0) * PHILOX_OPS
SW_BYTES_PER_SITE = 4.0 + 4.0 + (1.5 + 1.0 + 1.0) / 8.0
# 3D flip attempt: the 2D count plus one more threshold select (three
# thresholds for dE = 4J, 8J, 12J).
OPS_PER_FLIP_3D = OPS_PER_FLIP + 1


def cubic_leg(sweeps, warmup=10, rng=0):
    """3D sweeps of the 16 x 256^3 workload: flip attempts per second, the
    sweep kernel's roofline (derived ALU peak: the 2D instruction count per
    flip attempt plus one threshold select) and the oracle's rate on a bounded
    sample."""
    import torch

    import paper_2404_16990_amd as P
    import workloads

    w = workloads.cubic_16x256()
    descs = [dict(Lx=r.Lx, Ly=r.Ly, Lz=r.Lz, J=r.J, beta=r.beta, seed=r.seed, replica=r.replica, init=r.init,
                  rng=rng) for r in w.replicas]
    b = P.Batch3(descs)
    stream = b.stream
    b.run(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    b.run(sweeps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / sweeps
    b.close()
    flips = w.spins / (ms / 1e3)
    peak = lane_ops_peak() / OPS_PER_FLIP_3D
    # each sweep is two k3_sweep launches (one per colour) of half the sites
    out = {"workload": w.name, "spins": w.spins, "sweeps": sweeps, "rng": [k for k, v in RNG_NAMES.items() if v == rng][0],
           "value": flips, "unit": "flip attempts/s", "ms_per_sweep": ms,
           "roofline": {"bound": "alu", "kernel": "k3_sweep", "achieved": flips / 1e9, "peak": peak / 1e9,
                        "unit": "Gflip/s", "frac": flips / peak, "traffic": None, "launch_ms": ms / 2,
                        "per_unit": f"{OPS_PER_FLIP_3D} VALU instructions per flip attempt"}}
    from paper_2404_16990_amd import probe
    ceiling = probe.mix3_rate(rng=rng)
    out["roofline"]["measured_alu_ceiling"] = {
        "value": ceiling / 1e9, "unit": "Gflip/s", "frac": flips / ceiling,
        "kernel": f"k_mix3<rng={rng}> (the 3D per-word arithmetic on register-resident words)"}
    if rng == RNG_NAMES["bitsliced"]:
        ordered = probe.mix3_rate(rng=rng, bonds=1)
        out["roofline"]["measured_alu_ceiling_ordered_bonds"] = {
            "value": ordered / 1e9, "unit": "Gflip/s", "frac": flips / ordered,
            "kernel": f"k_mix3<rng={rng}, bonds=1> (neighbour words differing from the spin word in about "
                      f"11/32 of the bits)"}
    return out


def cubic_cpu_baseline(sweeps=2):
    import oracle
    import workloads
    w = workloads.cubic_16x256()
    descs = [oracle.desc3(r.Lx, r.Ly, r.Lz, r.J, r.beta, r.seed, r.replica, r.init) for r in w.replicas]
    states = [oracle.init_state3(d) for d in descs]
    threads = host_threads()
    t0 = time.perf_counter()
    oracle.run_batch3(descs, states, sweeps, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": w.spins * sweeps / dt, "unit": "flip attempts/s", "cores": threads, "kind": "oracle",
            "sample": f"all {len(w.replicas)} replicas x {sweeps} sweeps, {dt:.1f} s on {threads} host threads"}


def cluster_cpu_baseline(work, steps):
    """The CPU oracle's Swendsen-Wang steps on every replica of the workload."""
    import oracle
    descs = [oracle.desc(r.Lx, r.Ly, r.J, r.beta, r.seed, r.replica, r.init) for r in work.replicas]
    states = [oracle.init_state(d) for d in descs]
    threads = host_threads()
    t0 = time.perf_counter()
    oracle.run_cluster_batch(descs, states, steps, oracle.SWENDSEN_WANG, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": work.spins * steps / dt, "unit": "site updates/s", "cores": threads, "kind": "oracle",
            "sample": f"all {len(work.replicas)} replicas x {steps} SW steps, {dt:.1f} s on {threads} host threads"}


def cluster_leg(work, stream, steps, warmup=2):
    """Swendsen-Wang and Wolff steps of the workload's replicas: site updates
    per second (every step relabels every site) and the step's roofline."""
    import torch

    import paper_2404_16990_amd as P

    descs = [dict(Lx=r.Lx, Ly=r.Ly, J=r.J, beta=r.beta, seed=r.seed, replica=r.replica, init=r.init)
             for r in work.replicas]
    b = P.Batch(descs, stream=stream)
    out = {"workload": work.name, "steps": steps, "warmup": warmup,
           "metric": "site updates/s (a step labels every site; SW flips each cluster with prob. 1/2, "
                     "Wolff the cluster of one random site)"}
    for algo in ("sw", "wolff"):
        b.cluster(warmup, algo)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        b.cluster(steps, algo, 0)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        out[algo] = {"value": work.spins / (ms / 1e3), "unit": "site updates/s", "ms_per_step": ms}
    out["workspace_bytes"] = int(b.ws.numel())
    b.ws = None
    b.close()
    peak_alu = lane_ops_peak() / SW_OPS_PER_SITE
    peak_hbm = HBM_BYTES_PER_S / SW_BYTES_PER_SITE
    achieved = out["sw"]["value"]
    out["roofline"] = {
        "bound": "hbm" if peak_hbm <= peak_alu else "alu",
        "kernel": "k_cl_local + k_cl_cross<merge> + k_cl_cross<compress> + k_cl_flip (whole SW step)",
        "achieved": achieved / 1e9, "peak": min(peak_alu, peak_hbm) / 1e9, "unit": "Gsite/s",
        "frac": achieved / min(peak_alu, peak_hbm), "traffic": measured_cluster_traffic(work.name),
        "traffic_per": "one SW step (bytes); the counted bytes are " + f"{SW_BYTES_PER_SITE * work.spins:.4g}",
        "per_unit": f"{SW_OPS_PER_SITE:.1f} VALU instructions (0.5 + 1/128 Philox calls) and "
                    f"{SW_BYTES_PER_SITE:.2f} HBM bytes per site",
        "alu_peak": peak_alu / 1e9, "hbm_peak": peak_hbm / 1e9}
    return out


def critical_decorrelation(sw_steps, wolff_steps, plain_sweeps):
    """tau_int(|m|) and effective independent samples per second at T_c for
    Swendsen-Wang steps, Wolff steps and checkerboard Metropolis sweeps, on the
    64 replicas of 256^2 of the block-proposal workload (8 independent replicas
    at each of 8 temperatures; tau averaged over the 8 at T_c), equilibrated
    first by 2000 SW steps."""
    import numpy as np
    import torch

    import paper_2404_16990_amd as P
    from paper_2404_16990_amd import analysis, learned
    import workloads

    w = workloads.learned_64x256()
    descs = [dict(Lx=r.Lx, Ly=r.Ly, J=r.J, beta=r.beta, seed=r.seed, replica=r.replica, init=r.init)
             for r in w.replicas]
    b = P.Batch(descs)
    tc_group = [r for r in range(len(w.replicas)) if w.replicas[r].T == workloads.T_CRITICAL_PRINTED]
    b.cluster(2000, "sw")
    n = float(256 * 256)
    res = {"workload": w.name, "replicas_at_tc": tc_group, "T": workloads.T_CRITICAL_PRINTED}

    def summary(trace, seconds, units, unit_name):
        taus = np.array([analysis.tau_int(trace[r])[0] for r in tc_group])
        tau = float(taus.mean())
        rate = analysis.effective_rate(units / seconds, tau)
        return {f"tau_int_{unit_name}": tau, f"tau_int_{unit_name}_error": float(taus.std(ddof=1) / np.sqrt(len(taus))),
                unit_name: units, "seconds": seconds, "effective_samples_per_s": rate,
                "mean_abs_m": float(trace[tc_group].mean())}

    for algo, steps in (("sw", sw_steps), ("wolff", wolff_steps)):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(b.stream)
        _, mag = b.cluster(steps, algo, 1)
        e1.record(b.stream)
        torch.cuda.synchronize()
        tr = np.abs(mag.cpu().numpy().astype(np.float64)) / n
        res[algo] = summary(tr, e0.elapsed_time(e1) / 1e3, steps, "steps")
    tr_p, _, s_p = learned.plain_trace(b, plain_sweeps, 10)
    plain = summary(tr_p, s_p, plain_sweeps // 10, "points")
    plain["tau_int_sweeps"] = plain["tau_int_points"] * 10
    res["metropolis"] = plain
    for algo in ("sw", "wolff"):
        res[algo]["over_metropolis"] = res[algo]["effective_samples_per_s"] / plain["effective_samples_per_s"]
    b.ws = None
    b.close()
    return res


def roofline_of(m, work, rng_name):
    """Roofline object of the dominant kernel of a timed plain-path run."""
    from paper_2404_16990_amd import probe
    sched = m["schedule"]
    peak = alu_peak_flips()
    traffic, algo_bytes = (None, None)
    if rng_name == "site":
        kern = m["kernel"].split(" ")[0]
        spl = sched["sweeps_per_launch"] if m["kernel"] != "k_sweep_stream" else 0
        traffic, algo_bytes = measured_traffic(kern, work.name, spl)
    launch_s = m["launch_s"]
    roof = {"bound": "alu", "kernel": m["kernel"], "achieved": m["achieved"] / 1e9, "peak": peak / 1e9,
            "unit": "Gflip/s", "frac": m["achieved"] / peak, "traffic": traffic,
            "per_unit": f"{OPS_PER_FLIP} VALU instructions per flip attempt",
            "peak_basis": f"{CUS} CUs x {LANE_OPS_PER_CU_CLK} integer VALU lanes per clock x "
                          f"{CLOCK_HZ / 1e9:.1f} GHz = {lane_ops_peak():.3g} lane-ops/s / {OPS_PER_FLIP}",
            "launch_ms": launch_s * 1e3, "launches": m["launches"], "flips_per_launch": m["flips_per_launch"],
            "hbm_bytes_per_launch_algorithmic": algo_bytes,
            "hbm_frac_of_8TBps": (traffic / launch_s / HBM_BYTES_PER_S) if traffic else None}
    # measured ALU ceiling: the same per-word arithmetic with no memory traffic
    ceiling = probe.mix_rate(sched["word_bits"], rng=RNG_NAMES[rng_name])
    roof["measured_alu_ceiling"] = {
        "value": ceiling / 1e9, "unit": "Gflip/s",
        "frac": m["achieved"] / ceiling if ceiling >= m["achieved"] else None,
        "valid": bool(ceiling >= m["achieved"]),
        "kernel": f"k_mix<{sched['word_bits']}-bit, rng={rng_name}> (ising::update_word on two "
                  f"register-resident words per thread, best shape and launch)"}
    if rng_name == "bitsliced":
        # the lazy comparison's depth depends on how many sites are undecided:
        # the same probe with the bond statistics of an ordered 2D lattice
        ordered = probe.mix_rate(sched["word_bits"], rng=RNG_NAMES[rng_name], bonds=1)
        roof["measured_alu_ceiling_ordered_bonds"] = {
            "value": ordered / 1e9, "unit": "Gflip/s",
            "frac": m["achieved"] / ordered if ordered >= m["achieved"] else None,
            "valid": bool(ordered >= m["achieved"]),
            "kernel": f"k_mix<{sched['word_bits']}-bit, rng={rng_name}, bonds=1> (neighbour words differing "
                      f"from the spin word in about 1/8 of the bits)"}
    return roof


def config_leg(name, args, stream):
    """Another plain configuration timed like the headline (autotuned, the
    same steps and warm-up); returns its measurement and roofline."""
    import torch
    import workloads
    work = workloads.ALL[name]()
    m, b = run_path(work, 0, args, stream, json.loads(args.configs_schedule) if args.configs_schedule else None)
    out = {"workload": work.name, "replicas": len(work.replicas), "spins": work.spins,
           "value": m["value"], "unit": "flip attempts/s", "ms_per_step": m["ms_per_step"],
           "sweeps_per_step": args.sweeps_per_step, "steps": args.steps, "schedule": m["schedule"],
           "resident_replicas": m["resident_replicas"], "streamed_replicas": m["streamed_replicas"],
           "autotune": m["autotune"], "roofline": roofline_of(m, work, "site")}
    b.close()
    del b
    torch.cuda.empty_cache()
    return out


def headline(work, rng, args, stream):
    """The headline measurement: the workload under contract `rng`, timed;
    returns the JSON line's fields."""
    import torch
    m, batch = run_path(work, rng, args, stream, json.loads(args.schedule) if args.schedule else None)
    sched = m["schedule"]
    roofline = roofline_of(m, work, args.rng)
    out = {
        "metric": "aggregate flip attempts/s on 1 MI355X",
        "value": m["value"],
        "unit": "flip attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": work.name, "replicas": len(work.replicas), "spins": work.spins,
                   "sweeps_per_step": args.sweeps_per_step, "record_every": m["rec_every"],
                   "rng": args.rng, "schedule": sched,
                   "resident_replicas": m["resident_replicas"], "streamed_replicas": m["streamed_replicas"],
                   "autotune": m["autotune"], "wall_s": m["wall_s"]},
        "roofline": roofline,
    }
    batch.close()
    del batch
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--sweeps-per-step", type=int, default=100)
    ap.add_argument("--workload", default="uneven_512")
    ap.add_argument("--configs", default="batch_256x1024,paper_scale",
                    help="other plain configurations timed the same way (comma list, '' for none)")
    ap.add_argument("--configs-schedule", default="",
                    help="JSON dict of a fixed execution schedule for the configurations (no autotuning)")
    ap.add_argument("--rng", default="site", choices=list(RNG_NAMES),
                    help="random-number contract of the measured path (site: one Philox word per site; "
                         "bitsliced: transposed group words drawn lazily)")
    ap.add_argument("--no-variant", action="store_true",
                    help="skip the second measurement under the other random-number contract")
    ap.add_argument("--cpu-sweeps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--schedule", default="", help="JSON dict overriding the execution schedule")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-proposal comparison (64 x 256^2 near T_c)")
    ap.add_argument("--learned-units", type=int, default=60000)
    ap.add_argument("--learned-train-steps", type=int, default=2000,
                    help="Adam steps of the learned leg's training (fewer only to profile it)")
    ap.add_argument("--plain-sweeps", type=int, default=1000000)
    ap.add_argument("--tune-sweeps", type=int, default=100)
    ap.add_argument("--no-3d", action="store_true", help="skip the 3D (simple cubic) leg")
    ap.add_argument("--cubic-sweeps", type=int, default=200)
    ap.add_argument("--no-cluster", action="store_true",
                    help="skip the Swendsen-Wang / Wolff leg (throughput and tau_int at T_c)")
    ap.add_argument("--cluster-steps", type=int, default=20)
    ap.add_argument("--critical-steps", type=int, default=20000,
                    help="SW and Wolff steps of the T_c decorrelation comparison (0 skips it)")
    ap.add_argument("--critical-sweeps", type=int, default=400000,
                    help="Metropolis sweeps of the T_c decorrelation comparison")
    ap.add_argument("--skip-headline", action="store_true",
                    help="run only the other legs (for profiling them); the JSON line then has no headline")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(replicas would shard across GPUs with no communication).", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads

    t_start = time.perf_counter()

    def progress(what):
        # one line per finished leg on stderr (stdout carries only the JSON line)
        print(f"bench: {what} ({time.perf_counter() - t_start:.1f} s)", file=sys.stderr, flush=True)

    work = workloads.ALL[args.workload]()
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    rng = RNG_NAMES[args.rng]
    out = {}
    if not args.skip_headline:
        out = headline(work, rng, args, stream)
        progress("timed steps done")
    if not args.no_variant and not args.skip_headline:
        # the same workload under the other random-number contract (its own
        # oracle and parity tests), scheduled and timed the same way
        other = [k for k in RNG_NAMES if k != args.rng][0]
        mv, bv = run_path(work, RNG_NAMES[other], args, stream, json.loads(args.schedule) if args.schedule else None)
        rv = roofline_of(mv, work, other)
        out["variants"] = {f"rng_{other}": {
            "value": mv["value"], "ms_per_step": mv["ms_per_step"], "launch_ms": mv["launch_s"] * 1e3,
            "schedule": mv["schedule"], "autotune": mv["autotune"],
            "frac_of_derived_peak": rv["frac"], "measured_alu_ceiling": rv["measured_alu_ceiling"],
            "measured_alu_ceiling_ordered_bonds": rv["measured_alu_ceiling_ordered_bonds"]}}
        bv.close()
        del bv
        torch.cuda.empty_cache()
        progress("variant done")
    configs = [c for c in args.configs.split(",") if c]
    if configs:
        out["configs"] = {}
        for name in configs:
            out["configs"][name] = config_leg(name, args, stream)
            progress(f"config {name} done")
    if not args.no_cluster:
        cw = workloads.batch_256x1024()
        out["cluster"] = cluster_leg(cw, stream, args.cluster_steps)
        progress("cluster steps done")
        if not args.no_cpu_baseline:
            out["cluster"]["cpu_baseline"] = cluster_cpu_baseline(cw, 3)
        if args.critical_steps > 0:
            out["cluster"]["critical"] = critical_decorrelation(args.critical_steps, args.critical_steps,
                                                                args.critical_sweeps)
            progress("critical comparison done")
        torch.cuda.empty_cache()
    if not args.no_3d:
        out["cubic"] = cubic_leg(args.cubic_sweeps)
        vb = cubic_leg(args.cubic_sweeps, rng=RNG_NAMES["bitsliced"])
        out["cubic"]["variants"] = {"rng_bitsliced": {k: vb[k] for k in ("value", "ms_per_sweep")}}
        out["cubic"]["variants"]["rng_bitsliced"]["frac_of_derived_peak"] = vb["roofline"]["frac"]
        out["cubic"]["variants"]["rng_bitsliced"]["measured_alu_ceiling"] = vb["roofline"]["measured_alu_ceiling"]
        out["cubic"]["variants"]["rng_bitsliced"]["measured_alu_ceiling_ordered_bonds"] = \
            vb["roofline"]["measured_alu_ceiling_ordered_bonds"]
        if not args.no_cpu_baseline:
            out["cubic"]["cpu_baseline"] = cubic_cpu_baseline()
        torch.cuda.empty_cache()
        progress("3D legs done")
    if not args.no_learned:
        out["learned"] = learned_comparison(args.learned_units, args.plain_sweeps, args.learned_train_steps)
        torch.cuda.empty_cache()
        progress("learned comparison done")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(work, args.cpu_sweeps, rng)
        progress("CPU baseline done")
    print(json.dumps(out), flush=True)


def learned_comparison(units, plain_sweeps, train_steps=2000):
    """Effective independent |m| samples per second at T_c: plain checkerboard
    sweeps against learned 8x8 block proposals (1 block round : 1 sweep).

    64 replicas of 256^2: 8 independent replicas at each of 8 temperatures in
    [2.20, 2.35], one of them T_c; tau_int at T_c is the mean over its 8
    replicas.  10^5 sweeps of burn-in, 98 x 16 x 64 = 100,352 training blocks
    taken 100 sweeps apart, 2000 Adam steps of 512 blocks; then a plain run
    and a learned run from the equilibrated state.  The two samplers'
    observables are compared per temperature with errors from the spread
    between the independent replicas.
    """
    import numpy as np
    import torch

    import paper_2404_16990_amd as P
    from paper_2404_16990_amd import learned
    import workloads

    w = workloads.learned_64x256()
    descs = [dict(Lx=r.Lx, Ly=r.Ly, J=r.J, beta=r.beta, seed=r.seed, replica=r.replica, init=r.init)
             for r in w.replicas]
    b = P.Batch(descs)
    groups = [[r for r in range(len(w.replicas)) if w.replicas[r].T == T] for T in workloads.LEARNED_TEMPS]
    tc_group = groups[workloads.LEARNED_TEMPS.index(workloads.T_CRITICAL_PRINTED)]
    b.run(100000)
    X, BN, K = learned.collect_blocks(b, 8, 16, 98, 100)
    net = P.Net(workloads.nn_initial_params(64), block=8, max_batch=512, max_seq=65536)
    t0 = time.perf_counter()
    hist = learned.train(net, X, BN, K, train_steps, 512, 2e-3, log_every=500)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    tr_p, e_p, s_p = learned.plain_trace(b, plain_sweeps, 10)
    acc = torch.zeros(len(descs), dtype=torch.int64, device="cuda")
    tr_l, e_l, s_l = learned.unit_traces(b, units, learned.learned_units(b, net, 0, acc), progress=5000)
    plain = learned.summarise(tr_p, s_p, 10, tc_group)
    plain["tau_int_sweeps"] = plain["tau_int_points"] * 10
    lrn = learned.summarise(tr_l, s_l, 1, tc_group)
    # per temperature, errors from the spread between independent replicas
    z = learned.replica_agreement(tr_p, tr_l, groups)
    ze = learned.replica_agreement(e_p, e_l, groups)
    # per replica with Sokal-window errors: a diagnostic, reliable only where
    # the run is many tau long
    zs = learned.agreement(tr_p, tr_l)
    zes = learned.agreement(e_p, e_l)
    # matrix-core work: per sequence and site, 3 layers x 10 K-steps x 4 channel
    # slices of a 16x16x32 BF16 tile shared by 16 sequences; per unit, a scored
    # and a sampled sequence for every block of the batch
    blocks = len(descs) * (256 // 8) * (256 // 8)
    flop_unit = 2 * blocks * 64 * (3 * 10 * 4 * 16 * 16 * 32 * 2 / 16)
    flop_train_step = 9 * 2.0 * 512 * 64 * 64 * 320
    return {
        "metric": "effective independent |m| samples/s at T_c (per replica, tau the mean over the 8 replicas "
                  "at T_c, whole-batch time)",
        "workload": w.name, "replicas_at_tc": tc_group, "T": workloads.T_CRITICAL_PRINTED,
        "training": {"blocks": int(X.shape[0]), "steps": train_steps, "batch": 512, "lr": 2e-3,
                     "loss": hist, "seconds": t_train},
        "plain": plain, "learned": lrn,
        "block_acceptance": float(acc.cpu().sum()) / (units * len(descs) * 1024),
        "roofline": {"bound": "mfma", "kernel": "k_nn_score + k_nn_sample (whole unit time)",
                     "achieved": flop_unit * units / s_l / 1e12, "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": flop_unit * units / s_l / 2.5e15, "traffic": None,
                     "per_unit": f"{flop_unit / 1e9:.1f} GFLOP of BF16 MFMA per unit"},
        "training_tflops": flop_train_step * train_steps / t_train / 1e12,
        "learned_over_plain": lrn["effective_samples_per_s"] / plain["effective_samples_per_s"],
        "agreement_errors": "per temperature, spread of the 8 independent replicas' run means (Student t, "
                            "about 14 degrees of freedom: 93.5 % of |z| < 2 expected)",
        "temperatures": list(workloads.LEARNED_TEMPS),
        "energy_agreement": dict(learned.agreement_summary(ze), z=[round(float(v), 3) for v in ze],
                                 per_replica_sokal=learned.agreement_summary(zes)),
        "abs_m_agreement": dict(learned.agreement_summary(z), z=[round(float(v), 3) for v in z],
                                per_replica_sokal=learned.agreement_summary(zs)),
        "run_over_tau": {"plain": plain["run_over_tau"], "learned": lrn["run_over_tau"]},
    }


if __name__ == "__main__":
    main()
