"""Builds the library in-tree with hipcc for gfx950, in three variants:

  libmpik.so          the release build;
  libmpik_check.so    the debug build with kernel bounds checks (-DMPIK_CHECK:
                      a failed check sets the problem's check word and skips
                      the access; mpi_plan_check reads the words);
  libmpik_hostsan.so  the host code under AddressSanitizer and
                      UndefinedBehaviorSanitizer, the device code as released
                      (for the CPU tests of the plan sizing and argument
                      checks, run with the sanitizer runtime preloaded).

    python -m paper_2505_22797_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libmpik.so")
LIB_CHECK = os.path.join(PKG, "libmpik_check.so")
LIB_HOSTSAN = os.path.join(PKG, "libmpik_hostsan.so")
SOURCES = [os.path.join(PKG, "csrc", "mpik.hip")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-shared", "-std=c++17",
    # packed FP32 vector instructions stay off in every HIP build
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


# sanitizers for the host compilation only (each flag scoped with -Xarch_host);
# the device code is the release code
HOSTSAN_FLAGS = [
    "-shared-libasan", "-Xarch_host", "-g", "-Xarch_host", "-fno-omit-frame-pointer",
    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-sanitize-recover=all",
]


def asan_runtime() -> str:
    """The shared AddressSanitizer runtime that libmpik_hostsan.so links to
    (preload it into the process that loads that library)."""
    res = subprocess.run([hipcc(), "--print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = res.stdout.strip()
    if res.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError("the AddressSanitizer runtime was not found")
    return path


def _variants():
    inc = "-I" + os.path.join(ROOT, "include")
    base = [hipcc(), *HIPCC_FLAGS, inc]
    hostsan = [hipcc(), *HIPCC_FLAGS, *HOSTSAN_FLAGS, inc]
    return [(LIB, base), (LIB_CHECK, base + ["-DMPIK_CHECK"]), (LIB_HOSTSAN, hostsan)]


def build(verbose: bool = False) -> str:
    """Compiles the three variants side by side; returns the release path."""
    procs = []
    for out, cmd in _variants():
        tmp = out + ".tmp"
        procs.append((out, tmp, subprocess.Popen(cmd + ["-o", tmp, *SOURCES], stdout=subprocess.PIPE,
                                                 stderr=subprocess.PIPE, text=True)))
    failed = []
    for out, tmp, p in procs:
        so, se = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(so + se)
            failed.append(os.path.basename(out))
        else:
            if verbose:
                sys.stderr.write(se)
            os.replace(tmp, out)
    if failed:
        raise RuntimeError("hipcc failed building " + ", ".join(failed))
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
