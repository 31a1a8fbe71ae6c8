"""The host runtime under AddressSanitizer and UndefinedBehaviorSanitizer.

A second copy of libdpmt is linked with its host code (context, validation,
FP64 decomposition, CP fits, rank selection, threshold fit, planning, operand
packing) built with -fsanitize=address,undefined (host side only; the
kernels' object is the normal one), and the host-only C ABI tests
(tests/test_abi_cpu.py: device = -1 contexts, no GPU calls) run against it in
a child process with the ASan runtime preloaded.  Any ASan report or UBSan
finding aborts that process, and the test fails."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.slow


def test_host_only_abi_tests_pass_under_asan_and_ubsan(tmp_path):
    from paper_1707_03268_amd import build
    lib = build.build_host_sanitized(str(tmp_path))
    syms = subprocess.run(["nm", "-D", lib], capture_output=True, text=True).stdout
    assert "__asan_report" in syms and "__ubsan_handle" in syms, "the copy is not instrumented"
    env = dict(os.environ)
    env.update({"DPMT_LIBRARY": lib, "LD_PRELOAD": build.asan_runtime(),
                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
                "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"})
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_abi_cpu.py"),
                        "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out
