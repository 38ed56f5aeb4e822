"""The library's host-side plan logic (geometry, ring blocking, FFT pass
plans, GEMM work lists, argument checks) run under AddressSanitizer through
the C ABI's host-only dry runs, on every workload and precision form:
tests/asan/plan_checks (built by __graft_entry__.build() via
tests/asan/build.py; host code instrumented, no kernel launched)."""
import os
import subprocess

import pytest

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "asan", "_build", "plan_checks")


def test_host_plan_logic_under_address_sanitizer():
    if not os.path.exists(EXE):
        pytest.fail(f"{EXE} is not built (run __graft_entry__.build())")
    env = dict(os.environ, ASAN_OPTIONS="abort_on_error=0:exitcode=23")
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.returncode, r.stdout[-2000:], r.stderr[-4000:])
    assert "0 failures" in r.stdout
