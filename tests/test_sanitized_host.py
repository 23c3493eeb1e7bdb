"""The library's host code built under AddressSanitizer and
UndefinedBehaviorSanitizer (device code unchanged), loaded into a child
process with the ASan runtime preloaded, runs the C-ABI tests clean: argument
checks, error strings, NULL handling and object lifetimes with no device."""

import os
import shutil
import subprocess
import sys

import pytest

from paper_2106_03172_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _stale(lib):
    if not os.path.exists(lib):
        return True
    t = os.path.getmtime(lib)
    return any(os.path.getmtime(os.path.join(B.CSRC, f)) > t for f in os.listdir(B.CSRC))


@pytest.fixture(scope="module")
def sanitized():
    if shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("hipcc not available")
    if _stale(B.SANITIZED_LIB):
        B.build(sanitize=True)
    return B.SANITIZED_LIB, B.sanitizer_runtime()


def test_sanitized_library_is_instrumented(sanitized):
    lib, _ = sanitized
    nm = shutil.which("nm")
    if nm is None:
        pytest.skip("nm not available")
    syms = subprocess.run([nm, "-D", "--undefined-only", lib], capture_output=True, text=True, check=True).stdout
    assert "__asan_" in syms and "__ubsan_handle_" in syms


def test_abi_tests_run_clean_under_asan_and_ubsan(sanitized):
    lib, rt = sanitized
    env = dict(os.environ, LD_PRELOAD=rt, SVR_LIBRARY=lib,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_abi.py"), "-q",
                        "-p", "no:cacheprovider", "-m", "not gpu"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in r.stdout
    # the child really mapped the sanitized library
    probe = ("import paper_2106_03172_amd as p; p.lib(); "
             "print(any(l.rstrip().endswith(%r) for l in open('/proc/self/maps')))" % lib)
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == "True", r.stdout + r.stderr
