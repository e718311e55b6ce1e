"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU).

Builds every library source for the host only with both sanitizers
(paper_2503_23144_amd.build.build_sanitized), then runs
  * tests/host_checks.cpp: the workspace arena (random alloc/free patterns,
    coalescing, exhaustion) and the program parser, transforms and pool
    planner, including malformed programs;
  * tests/test_host_library.py against the sanitized library: argument
    checks, program texts, the derived operation lists executed with numpy,
    the workspace estimates;
and requires both to pass with no sanitizer report.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def sanitized():
    sys.path.insert(0, ROOT)
    from paper_2503_23144_amd import build
    lib = build.build_sanitized(extra_sources=[os.path.join(ROOT, "tests", "host_checks.cpp")], verbose=False)
    env = dict(os.environ)
    env["LD_PRELOAD"] = build.asan_runtime()
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["LRCC_LIBRARY"] = lib
    return lib, os.path.join(build.SAN_DIR, "host_checks"), env


def _clean(out):
    return "AddressSanitizer" not in out and "runtime error:" not in out and "LeakSanitizer" not in out


@pytest.mark.slow
def test_host_checks_under_sanitizers(sanitized):
    _, exe, env = sanitized
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "host checks passed" in out and _clean(out), out[-4000:]


@pytest.mark.slow
def test_host_library_tests_under_sanitizers(sanitized):
    lib, _, env = sanitized
    probe = ("import re; from paper_2503_23144_amd import lrcc; maps = open('/proc/self/maps').read(); "
             "print(lrcc.LIB_PATH, 'asan' if 'libclang_rt.asan' in maps else 'no-asan')")
    r = subprocess.run([sys.executable, "-c", probe], capture_output=True, text=True, env=env, cwd=ROOT, timeout=300)
    assert r.stdout.split()[-2:] == [lib, "asan"], r.stdout + r.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_host_library.py")],
                       capture_output=True, text=True, env=env, cwd=ROOT, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and _clean(out), out[-4000:]
