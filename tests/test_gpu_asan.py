"""The runtime's host code under AddressSanitizer (tests/asan/harness.cpp, built by
__graft_entry__.build()): every C ABI path the harness drives returns what it should and
no invalid host memory access occurs."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

HARNESS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "asan", "_build",
                       "fpd_asan_harness")


def test_runtime_host_code_under_address_sanitizer():
    print("[case] asan harness", flush=True)
    assert os.path.exists(HARNESS), "build the harness first (__graft_entry__.build())"
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=86")
    out = subprocess.run([HARNESS], capture_output=True, text=True, timeout=240, env=env)
    print(out.stdout[-2000:], flush=True)
    assert "AddressSanitizer" not in out.stderr, out.stderr[-4000:]
    assert out.returncode == 0, out.stderr[-4000:]
    assert "all calls returned as expected" in out.stdout
