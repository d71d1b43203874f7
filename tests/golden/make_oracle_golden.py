"""Write tests/golden/oracle_single64.json and oracle_single64_bitsliced.json
from the CPU oracle only.

Records the (B, M) trace of the 64x64 lattice at T = 2.269185 (seed 16990,
replica 0, random start, 1000 sweeps, every sweep) and a digest of its final
state, under the site and under the bit-sliced random-number contract, so
that any later change to the oracle's arithmetic shows up as a failing test.
Run: python tests/golden/make_oracle_golden.py
"""
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads  # noqa: E402


def compute(rng=0):
    w = workloads.single_64()
    r = w.replicas[0]
    d = oracle.desc(r.Lx, r.Ly, r.J, r.beta, r.seed, r.replica, r.init, rng=rng)
    s = oracle.init_state(d)
    init_digest = hashlib.sha256(s.tobytes()).hexdigest()
    b, m = oracle.sweeps(d, s, w.sweeps, record_every=w.record_every)
    return {
        "workload": w.name,
        "rng": rng,
        "init_sha256": init_digest,
        "final_sha256": hashlib.sha256(s.tobytes()).hexdigest(),
        "bond": [int(v) for v in b],
        "mag": [int(v) for v in m],
    }


if __name__ == "__main__":
    for rng, name in ((0, "oracle_single64.json"), (1, "oracle_single64_bitsliced.json")):
        out = os.path.join(HERE, name)
        with open(out, "w") as f:
            json.dump(compute(rng), f)
        print(out)
