"""The solver lifecycle on the GPU with the library's host code under
AddressSanitizer and UndefinedBehaviorSanitizer (device code as in
libhhlb.so): the driver tests/sanitize/solver_lifecycle.cpp in its GPU mode
runs the autotuner's candidate loop twice on one solver of 512 channels of
the batched workload, switches launch configurations back to back with
steps queued and no synchronisation by the caller, and destroys solvers
with work in flight, in the FP64, mixed FP32 and mixed BF16 forms.  Needs
the driver built beforehand (python tests/sanitize/build_sanitized.py, also
done by the CPU sanitizer test)."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
EXE = os.path.join(HERE, "sanitize", "_build", "solver_lifecycle")
CHANNELS = os.path.join(HERE, "sanitize", "_build", "channels512.txt")


def test_solver_lifecycle_under_host_sanitizers():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not (os.path.exists(EXE) and os.path.exists(CHANNELS)):
        pytest.skip("sanitized driver not built (python tests/sanitize/build_sanitized.py)")
    root = os.path.dirname(HERE)
    csrc = os.path.join(root, "paper_1708_03249_amd", "csrc")
    sources = [os.path.join(HERE, "sanitize", "solver_lifecycle.cpp"), os.path.join(root, "include", "hhlb.h")]
    sources += [os.path.join(csrc, f) for f in os.listdir(csrc) if f.endswith((".hip", ".hpp", ".cpp", ".h"))]
    stale = [f for f in sources if os.path.getmtime(f) > os.path.getmtime(EXE)]
    if stale:
        pytest.skip(f"sanitized driver older than {os.path.basename(stale[0])}: rebuild it "
                    "(python tests/sanitize/build_sanitized.py)")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    print(f"[sanitize] {EXE} gpu {CHANNELS}", flush=True)
    r = subprocess.run([EXE, "gpu", CHANNELS], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                       env=env, timeout=300)
    print(r.stdout[-3000:], flush=True)
    assert r.returncode == 0, r.stdout[-3000:]
    assert "checks OK" in r.stdout
