"""Builds the HIP library ``_lib/libsvr.so`` for gfx950 with hipcc.

Every translation unit is compiled with floating-point contraction off
(results are the correctly rounded operations as written, so a quantity
computed by two kernels is bitwise identical) and with packed FP32
instructions disabled.

Usage: ``python -m paper_2106_03172_amd.build`` (or ``build()`` from Python).
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "_lib")
BUILDDIR = os.path.join(os.path.dirname(HERE), "_build")
LIB = os.path.join(LIBDIR, "libsvr.so")

SOURCES = ["util.hip", "geom.hip", "proj.hip", "update.hip", "persist.hip", "slices.hip", "api.hip", "serve.hip", "tune.hip",
           "batch.hip"]
ARCH = os.environ.get("SVR_OFFLOAD_ARCH", "gfx950")
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # a kernel's leading scalar and pointer arguments arrive in SGPRs at wave
    # launch, so its first loads need not wait for the argument fetch (the code
    # object keeps a prologue that loads them where the firmware cannot preload)
    "-mllvm", "-amdgpu-kernarg-preload-count=16",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
]

# roctx ranges around the host phases (csrc/trace.h)
LINK = ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]


def _hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(c) or c == "hipcc":
            return c
    raise RuntimeError("hipcc not found")


# AddressSanitizer and UndefinedBehaviorSanitizer for the host code only (the
# device code is built as always).  The library then expects the ASan runtime
# to be preloaded into the process (``sanitizer_runtime()``).
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
SANITIZED_LIB = os.path.join(BUILDDIR, "sanitize", "libsvr.so")


def sanitizer_runtime() -> str:
    """Path of the compiler's shared ASan runtime (it also carries the UBSan
    handlers) that a process preloads to run the sanitized library."""
    r = subprocess.run([_hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError("ASan runtime not found")
    return path


def _compile(src: str, defines=(), builddir=BUILDDIR, extra=()) -> str:
    obj = os.path.join(builddir, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), *FLAGS, *extra, *[f"-D{d}" for d in defines], "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    warn = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if "warning" in warn:
        sys.stderr.write(warn + "\n")
    return obj


def build(verbose: bool = False, defines=(), out: str = LIB, sanitize: bool = False) -> str:
    """Compiles every source and links the shared library; returns its path.
    ``defines`` (e.g. ``["SVR_BP_G=8"]``) override the kernels' tuning constants;
    ``sanitize`` builds the host code under ASan and UBSan into its own folder
    (``SANITIZED_LIB`` unless ``out`` says otherwise)."""
    builddir = BUILDDIR if not defines else os.path.join(BUILDDIR, "_".join(defines).replace("=", ""))
    extra = ()
    if sanitize:
        builddir = os.path.join(builddir, "sanitize")
        extra = SANITIZE
        if out == LIB:
            out = SANITIZED_LIB
    os.makedirs(builddir, exist_ok=True)
    os.makedirs(os.path.dirname(out), exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, defines, builddir, extra), srcs))
    tmp = out + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, *LINK]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    build(verbose=True, sanitize="--sanitize" in sys.argv[1:])
