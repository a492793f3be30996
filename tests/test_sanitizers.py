"""The server's host code under sanitizers, on the CPU: the stress driver
(tests/native/server_stress.cpp: concurrent submitters and waiters,
cancellation racing the scheduler, an injected device failure, destruction
with work queued, chunked and waited on) against a library whose host code is
built with AddressSanitizer + UndefinedBehaviorSanitizer, and with
ThreadSanitizer.  Any report aborts the driver.  The builds are cached under
_build/ by a hash of the sources."""
import hashlib
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2606_01547_amd", "csrc")
OUT = os.path.join(ROOT, "_build", "sanitized")
DRIVER = os.path.join(ROOT, "tests", "native", "server_stress.cpp")

pytestmark = pytest.mark.slow


def _sources_hash():
    h = hashlib.sha256()
    files = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                   if f.endswith((".hip", ".cpp", ".hpp", ".inc", ".sh")))
    for f in files + [DRIVER, os.path.join(ROOT, "include", "jt.h")]:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def _build(kind):
    if not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("no HIP toolchain")
    stamp = os.path.join(OUT, f"{kind}.stamp")
    want = _sources_hash()
    exe = os.path.join(OUT, f"server_stress_{kind}")
    if not (os.path.exists(exe) and os.path.exists(stamp) and open(stamp).read() == want):
        subprocess.run(["sh", os.path.join(CSRC, "build_sanitized.sh"), kind, OUT], check=True,
                       capture_output=True, timeout=600)
        with open(stamp, "w") as f:
            f.write(want)
    return exe


@pytest.mark.parametrize("kind,env", [
    ("asan", {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=1",
              "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}),
    ("tsan", {"TSAN_OPTIONS": "halt_on_error=1:second_deadlock_stack=1"}),
])
def test_server_stress_under_sanitizer(kind, env):
    exe = _build(kind)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env={**os.environ, **env})
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "Sanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert "destroy with work pending: ok" in r.stdout
