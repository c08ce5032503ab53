"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The sanitized build (paper_1506_06513_amd.build.build_sanitized) instruments
the host side of every unit with -fsanitize=address,undefined; the paths in
tests/asan_host_paths.py run in a subprocess with the ASan runtime preloaded
and must finish without a sanitizer report.  The test builds the library
when it is missing or older than the sources.  It runs on the CPU only: the
ROCm ASan runtime also intercepts the HIP runtime's device-memory pool
allocations (its GPU-sanitizer hooks) and fails them on a device without
that support, so device runs under it are not meaningful here."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
from paper_1506_06513_amd import build as B  # noqa: E402

SCRIPT = os.path.join(ROOT, "tests", "asan_host_paths.py")


def _run(*args):
    env = dict(os.environ)
    env["LD_PRELOAD"] = B.asan_runtime()
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([sys.executable, SCRIPT, *args], capture_output=True, text=True, env=env, timeout=600)
    report = [l for l in (r.stdout + r.stderr).splitlines()
              if "AddressSanitizer" in l or "runtime error:" in l or "UndefinedBehaviorSanitizer" in l]
    assert not report, "\n".join(report[:20] + (r.stdout + r.stderr).splitlines()[-30:])
    assert r.returncode == 0, (r.stdout + r.stderr)[-3000:]
    return r.stdout


def test_host_paths_under_asan_and_ubsan():
    if not B.sanitized_current():
        B.build_sanitized()
    assert "host paths: ok" in _run()

