"""The host-only code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU): the oracle, the input generator, the int32 packer, the serving
scheduler on its simulated clock, the tuning-cache parser and the ABI's
argument checks, driven by tests/sanitize/host_checks.cpp.  Any sanitizer
report aborts the driver, so the test fails."""
import os
import subprocess
import sys
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.slow
def test_host_code_under_sanitizers():
    sys.path.insert(0, os.path.join(HERE, "sanitize"))
    import build as sanitize_build
    binary = sanitize_build.build()
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1",
               HIP_VISIBLE_DEVICES="")          # host code only: no device, whatever the machine has
    env.pop("AGG_FAULT_INJECT", None)
    with tempfile.TemporaryDirectory() as d:
        r = subprocess.run([binary, d], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0 and "host checks ok" in r.stdout, (r.stdout[-2000:] + r.stderr[-6000:])
