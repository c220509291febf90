"""The C ABI from a plain C program (tests/c/abi_cycle.c, built by build()).

The program allocates device memory through the HIP runtime, builds the
1000-node cycle from CSR arrays, applies the heat kernel and runs Algorithm 1,
and checks them against the cycle's closed forms (see its header comment).
It runs as a child process, so no Python or torch is involved in its calls.
"""
import os
import subprocess

import pytest

from gpu_common import need_gpu

pytestmark = pytest.mark.gpu
BIN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c", "abi_cycle")


def test_plain_c_client():
    need_gpu()
    if not os.path.exists(BIN):
        pytest.fail("tests/c/abi_cycle is not built (run __graft_entry__.build())")
    r = subprocess.run([BIN], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    assert "abi_cycle ok" in r.stdout, r.stdout
