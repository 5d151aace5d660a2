"""The host core (code construction, planning, the C ABI's host functions)
under AddressSanitizer and UndefinedBehaviorSanitizer (the host parity and
thread suites against libbpx_san.so) and under ThreadSanitizer (the thread
suite against libbpx_tsan.so), each in a child process with the sanitizer
runtime preloaded; any report fails the test.  CPU only."""
import os
import subprocess
import sys

import pytest

from conftest import ROOT


@pytest.mark.slow
def test_host_parity_under_asan_ubsan():
    from paper_1904_11563_amd import build
    lib = build.build_sanitized()
    rt = build.sanitizer_runtime()
    if not os.path.exists(rt):
        pytest.skip("no shared AddressSanitizer runtime next to hipcc")
    env = dict(os.environ)
    env.update({"LD_PRELOAD": rt, "BPX_LIBRARY": lib,
                "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=1",
                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"})
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_host_parity.py"),
                        os.path.join(ROOT, "tests", "test_host_threads.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    reports = [l for l in out.splitlines() if "Sanitizer" in l or "runtime error" in l]
    assert r.returncode == 0 and not reports, "\n".join(reports[:20]) or out[-3000:]
    assert "passed" in r.stdout


@pytest.mark.slow
def test_host_threads_under_tsan():
    from paper_1904_11563_amd import build
    lib = build.build_sanitized("thread")
    rt = build.sanitizer_runtime("thread")
    if not os.path.exists(rt):
        pytest.skip("no shared ThreadSanitizer runtime next to hipcc")
    env = dict(os.environ)
    env.update({"LD_PRELOAD": rt, "BPX_LIBRARY": lib, "TSAN_OPTIONS": "halt_on_error=1"})
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_host_threads.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    reports = [l for l in out.splitlines() if "ThreadSanitizer" in l and "Running" not in l]
    assert r.returncode == 0 and not reports, "\n".join(reports[:20]) or out[-3000:]
    assert "3 passed" in r.stdout

