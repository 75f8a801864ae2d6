"""The library's host code under AddressSanitizer, LeakSanitizer and
UndefinedBehaviorSanitizer (tests/sanitize/build_sanitized.py builds the
library's sources and the driver tests/sanitize/solver_lifecycle.cpp with
the sanitizers on the host side only).  Here, without a GPU, the driver's
host mode: the velocity sets, force matrices and equilibria of every model
kind, solvers for every kind of channel and for 512 channels of the batched
workload in each arithmetic form, the launch-configuration checks and the
argument-error paths, each checked for its status code."""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "sanitize"))


@pytest.fixture(scope="module")
def driver():
    if not (shutil.which("/opt/rocm/bin/hipcc") and os.path.exists("/opt/rocm/llvm/bin/clang++")):
        pytest.skip("no ROCm toolchain")
    import build_sanitized
    return build_sanitized.build(), build_sanitized.CHANNELS


def test_host_code_is_clean_under_sanitizers(driver):
    exe, channels = driver
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, "host", channels], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                       env=env, timeout=600)
    print(r.stdout[-3000:])
    assert r.returncode == 0, r.stdout[-3000:]
    assert "checks OK" in r.stdout
    assert "runtime error" not in r.stdout and "Sanitizer" not in r.stdout
