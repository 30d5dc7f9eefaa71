"""The C-ABI driven from plain C (tests/abi_c/abi_check.c): device memory
from hipMalloc, no Python binding.  The program checks constant-state
preservation through hwenou_advance (1D and 2D Euler, FP64 and mixed,
periodic, outflow and wall sides) and argument errors of hwenou_stage and
hwenou_create; it is built by __graft_entry__.build()."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(__file__), "abi_c", "abi_check")


def test_c_caller():
    print("[gpu] plain-C caller of the C-ABI", flush=True)
    assert os.path.exists(EXE), "build it first: python -c 'import __graft_entry__ as g; g.build()'"
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0 and "abi_check: ok" in r.stdout
