"""Build the standalone C program that drives libising.so through its C ABI
with the HIP runtime API only (tests/c/abi_standalone, run by a GPU test).
Needs the library built first (paper_2404_16990_amd/_lib/libising.so)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
SRC = os.path.join(HERE, "abi_standalone.c")
OUT = os.path.join(HERE, "abi_standalone")


def build(verbose=False):
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-Werror",
           # the HIP runtime header, used from a plain C compiler, needs the platform named
           "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include"), "-I", os.path.join(ROOT, "include"),
           SRC, "-L", os.path.join(ROOT, "paper_2404_16990_amd", "_lib"), "-lising",
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-lm",
           "-Wl,-rpath,$ORIGIN/../../paper_2404_16990_amd/_lib", "-Wl,-rpath," + os.path.join(ROCM, "lib"),
           "-o", OUT + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("building the C ABI program failed:\n" + r.stderr)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
