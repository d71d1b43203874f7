"""Build the C oracle (test infrastructure: 2D sweeps, cluster steps, 3D sweeps) into
oracle/liboracle.so with gcc.

Run as ``python oracle/build.py``.  The GPU library never links this file's
output; it is compiled only so that tests and the benchmark's CPU-baseline leg
can load it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "ising_oracle.c"), os.path.join(HERE, "cluster_oracle.c"),
        os.path.join(HERE, "ising3d_oracle.c")]
OUT = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=c99", "-O2", "-fPIC", "-shared", "-pthread", "-Wall", "-Wextra",
           "-o", OUT + ".tmp", *SRCS, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
