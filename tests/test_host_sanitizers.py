"""The host code of the library -- plan sizing, descriptor and argument
checks, the allocation-failure hook -- under AddressSanitizer and
UndefinedBehaviorSanitizer: tests/test_abi_cpu.py runs in a child process
against libmpik_hostsan.so (host code only, built with both sanitizers and no
recovery) with the sanitizer runtime preloaded.  CPU only: the child makes no
device call."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOSTSAN = os.path.join(ROOT, "paper_2505_22797_amd", "libmpik_hostsan.so")


def test_abi_tests_pass_under_asan_and_ubsan():
    if not os.path.exists(HOSTSAN):
        pytest.skip("libmpik_hostsan.so is not built")
    if os.environ.get("LD_PRELOAD"):
        pytest.skip("another library is preloaded; the sanitizer runtime has to come first")
    from paper_2505_22797_amd import build as B
    env = dict(os.environ)
    env["LD_PRELOAD"] = B.asan_runtime()
    # the interpreter and torch are not instrumented: leaks and allocator
    # mismatches there are not the library's
    env["ASAN_OPTIONS"] = "detect_leaks=0:alloc_dealloc_mismatch=0:detect_odr_violation=0:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["MPIK_LIBRARY"] = "libmpik_hostsan.so"
    env["HIP_VISIBLE_DEVICES"] = ""
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                          os.path.join(ROOT, "tests", "test_abi_cpu.py")],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-6000:]
    assert "passed" in res.stdout
    for marker in ("ERROR: AddressSanitizer", "runtime error:", "SUMMARY: UndefinedBehaviorSanitizer"):
        assert marker not in out, out[-6000:]
