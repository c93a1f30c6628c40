"""The C ABI's host code under AddressSanitizer: the driver built beside the
library (host code compiled with -fsanitize=address, see build.py) drives
every documented error path of the entry points with malformed descriptions
and options, and runs a small segment batch (forward and backward, both
schedules, LDS poisoning on), a cut, a graph and an MPC build end to end.
An out-of-bounds host access aborts it; a wrong error code fails a check."""
import os
import subprocess

import pytest

from paper_2411_13507_amd import build

pytestmark = pytest.mark.gpu


def test_abi_checks_under_address_sanitizer(gpu_available):
    if not os.path.exists(build.ABI_CHECK):
        pytest.skip("AddressSanitizer build of the ABI check not present (no g++ where the library was built)")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")   # the HIP runtime keeps its allocations to exit
    print("case: ABI checks under AddressSanitizer", flush=True)
    r = subprocess.run([build.ABI_CHECK], capture_output=True, text=True, timeout=120, env=env)
    print(r.stdout[-4000:], r.stderr[-4000:])
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "PASSED" in r.stdout and "FAIL " not in r.stdout
