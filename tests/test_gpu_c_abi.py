"""The C ABI from plain C: tests/c/abi_standalone (built by build() of the
repository entry point) creates, runs and reads a batch with the HIP runtime
API only and checks exact properties (see its header); it runs here as a child
process."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c", "abi_standalone")


def test_c_program_drives_the_library():
    assert os.path.exists(EXE), "tests/c/abi_standalone is not built (run __graft_entry__.build())"
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", (r.returncode, r.stdout, r.stderr)
