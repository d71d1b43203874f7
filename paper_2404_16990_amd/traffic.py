"""HBM traffic per launch from rocprofv3 counter runs (a measurement helper).

Reads the counter_collection CSVs of two ``rocprofv3 --pmc`` runs of a
program (one with FETCH_SIZE, one with WRITE_SIZE; KiB per dispatch) and the
same two counters for the probe library's plain copy kernel of known size,
scales each counter by copy bytes / counter reading, and writes the JSON
summary bench.py reads for the ``traffic`` field of its roofline object.

A "launch" may be a unit of several dispatches (for a mixed schedule: 2 S
streaming launches and one resident launch per chunk of S sweeps); --part
gives each kernel (a substring of its name) and how many of its dispatches one
unit holds.

Usage (repository root, after the four counter runs):

    python -m paper_2404_16990_amd.traffic --fetch DIR --write DIR --copy-fetch DIR --copy-write DIR \\
        --copy-bytes 268435456 --part 'k_sweep_stream<unsigned long, 256>=100' \\
        --part 'k_sweep_resident<unsigned long, 1024>=1' --kernel k_sweep_stream --workload NAME \\
        --sweeps-per-launch 50 --algorithmic-bytes B --command '...' --out profiles/traffic_....json
"""
import argparse
import csv
import glob
import json
import os
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def per_dispatch(directory, counter, match):
    """Mean over dispatches whose kernel name contains `match` of the counter's
    value summed over its rows (one dispatch may report several dimensions)."""
    files = glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {directory}")
    sums = defaultdict(float)
    for path in files:
        with open(path) as f:
            for row in csv.DictReader(f):
                if row["Counter_Name"] != counter or match not in row["Kernel_Name"]:
                    continue
                sums[(path, row["Dispatch_Id"])] += float(row["Counter_Value"])
    if not sums:
        raise ValueError(f"no {counter} rows for kernels matching {match!r} under {directory}")
    return sum(sums.values()) / len(sums), len(sums)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-fetch", required=True)
    ap.add_argument("--copy-write", required=True)
    ap.add_argument("--copy-bytes", type=int, required=True, help="bytes the copy kernel reads (and writes)")
    ap.add_argument("--part", action="append", required=True, help="KERNEL_SUBSTRING=DISPATCHES_PER_UNIT")
    ap.add_argument("--kernel", required=True, help="kernel label stored in the summary")
    ap.add_argument("--workload", required=True)
    ap.add_argument("--sweeps-per-launch", type=int, required=True, help="0 for per-colour streaming launches")
    ap.add_argument("--algorithmic-bytes", type=float, required=True, help="algorithmic HBM bytes per unit")
    ap.add_argument("--command", action="append", default=[], help="commands that produced the counter runs")
    ap.add_argument("--out", required=True)
    args = ap.parse_args()

    import sys
    sys.path.insert(0, ROOT)
    import bench

    cf, _ = per_dispatch(args.copy_fetch, "FETCH_SIZE", "k_copy")
    cw, _ = per_dispatch(args.copy_write, "WRITE_SIZE", "k_copy")
    fetch_scale = args.copy_bytes / (cf * 1024.0)
    write_scale = args.copy_bytes / (cw * 1024.0)
    parts, fetch_kib, write_kib, traffic = [], 0.0, 0.0, 0.0
    for spec in args.part:
        name, mult = spec.rsplit("=", 1)
        mult = float(mult)
        f, nf = per_dispatch(args.fetch, "FETCH_SIZE", name)
        w, nw = per_dispatch(args.write, "WRITE_SIZE", name)
        parts.append({"kernel": name, "dispatches_per_unit": mult, "fetch_size_kib_per_dispatch": f,
                      "write_size_kib_per_dispatch": w, "dispatches": [nf, nw]})
        fetch_kib += mult * f
        write_kib += mult * w
        traffic += mult * (f * fetch_scale + w * write_scale) * 1024.0
    entry = {"fetch_size_kib_per_unit": fetch_kib, "write_size_kib_per_unit": write_kib,
             "traffic_bytes_per_launch": traffic, "algorithmic_bytes_per_launch": args.algorithmic_bytes,
             "parts": parts, "commands": args.command}
    out = {}
    if os.path.exists(args.out):
        with open(args.out) as f:
            out = json.load(f)
        if out.get("kernel_source_sha256") != bench.kernel_source_digest():
            out = {}
    out.update({
        "kernel": args.kernel,
        "workload": args.workload,
        "kernel_source_sha256": bench.kernel_source_digest(),
        "kernel_sources": ["paper_2404_16990_amd/csrc/kernels.hip", "paper_2404_16990_amd/csrc/device.hpp",
                           "paper_2404_16990_amd/csrc/launch.hpp"],
        "copy_calibration": {"bytes_each_way": args.copy_bytes, "fetch_size_kib": cf, "write_size_kib": cw,
                             "fetch_scale": fetch_scale, "write_scale": write_scale},
        "algorithmic_bytes_per_launch": args.algorithmic_bytes,
    })
    out.setdefault("by_sweeps_per_launch", {})[str(args.sweeps_per_launch)] = entry
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({"traffic_bytes_per_launch": traffic, "algorithmic": args.algorithmic_bytes,
                      "ratio": traffic / args.algorithmic_bytes}))


if __name__ == "__main__":
    main()
