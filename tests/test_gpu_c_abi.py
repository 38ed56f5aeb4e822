"""The C ABI from C alone: tests/c_abi/roundtrip.c (built by
__graft_entry__.build() against the in-tree libshtx.so) creates a plan,
allocates with the HIP runtime, runs one inverse and one direct transform
and checks them against the closed forms of P̄_1^0 and P̄_1^1 fields."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi", "_build", "roundtrip")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_c_program_roundtrip(prec):
    if not os.path.exists(EXE):
        pytest.fail(f"{EXE} is not built (run __graft_entry__.build())")
    r = subprocess.run([EXE, prec], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
