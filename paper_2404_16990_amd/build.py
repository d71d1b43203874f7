"""Compile the HIP library for gfx950 into paper_2404_16990_amd/_lib/libising.so.

Run as ``python -m paper_2404_16990_amd.build``.  Always recompiles.
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT_DIR = os.path.join(PKG, "_lib")
OUT = os.path.join(OUT_DIR, "libising.so")
SOURCES = ["kernels.hip", "api.cpp", "nn.hip", "nn_api.cpp", "cluster.hip", "cluster_api.cpp", "ising3d.hip",
           "ising3d_api.cpp"]
PROBE_OUT = os.path.join(OUT_DIR, "libising_probe.so")
PROBE_SOURCES = ["probe.hip"]
# Packed FP32 instructions stay disabled in every HIP build of this project.
# Matrix-core results go to ordinary vector registers (the VGPR form of the
# MFMA instructions), so the activations read them without a copy out of the
# accumulation registers.
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-mllvm", "-amdgpu-mfma-vgpr-form=1"]


def _compile(sources, out, verbose):
    cmd = ["hipcc", *HIP_FLAGS, "-shared", "-I", os.path.join(ROOT, "include"),
           *[os.path.join(CSRC, s) for s in sources], "-o", out + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in res.stderr.splitlines() if noise not in l)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + err)
    if err.strip() and verbose:
        print(err, file=sys.stderr)
    os.replace(out + ".tmp", out)
    return out


def build(verbose: bool = False) -> str:
    """Compile libising.so (the sweep library) and libising_probe.so (micro-benchmarks)."""
    os.makedirs(OUT_DIR, exist_ok=True)
    _compile(PROBE_SOURCES, PROBE_OUT, verbose)
    return _compile(SOURCES, OUT, verbose)


if __name__ == "__main__":
    print(build(verbose=True))
