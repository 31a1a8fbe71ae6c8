"""Build libdpmt.so in-tree with hipcc for gfx950.

    python -m paper_1707_03268_amd.build

Compiles the host runtime and the HIP kernels to objects under _build/ and
links them into one shared library next to this file.  Packed FP32
instructions are disabled for all device code.

build_host_sanitized() links a second copy whose host runtime is built with
AddressSanitizer and UndefinedBehaviorSanitizer (host code only; the kernels'
object is the normal one), for the CPU tests of the host-only paths.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdpmt.so")
BUILD_DIR = os.path.join(ROOT, "_build")
HOST_SRC = os.path.join(CSRC, "dpmt_host.cpp")
KERNEL_SRCS = [os.path.join(CSRC, "dpmt_kernels.hip"), os.path.join(CSRC, "dpmt_hog.hip")]
ARCH = "gfx950"
COMMON = ["-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function", "-Wno-unused-result"]
NOISE = "is not a recognized feature for this target"


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def _includes():
    return ["-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _run(cmd, verbose: bool) -> None:
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (res.stdout + res.stderr).splitlines() if NOISE not in l)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{msgs}")
    if verbose and msgs.strip():
        print(msgs)


def _object(src: str) -> str:
    return os.path.join(BUILD_DIR, os.path.splitext(os.path.basename(src))[0] + ".o")


def _compile_all(cmds, verbose: bool) -> None:
    """Run the compile commands side by side; raise on the first failure."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
        for f in [ex.submit(_run, cmd, verbose) for cmd in cmds]:
            f.result()


def _kernel_cmd(src: str):
    return [hipcc(), f"--offload-arch={ARCH}", "-O3", *COMMON, *_includes(), "-c", src, "-o", _object(src)]


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    hobj = os.path.join(BUILD_DIR, "dpmt_host.o")
    _compile_all([_kernel_cmd(s) for s in KERNEL_SRCS] +
                 [[hipcc(), f"--offload-arch={ARCH}", "-O3", *COMMON, *_includes(), "-c", HOST_SRC,
                   "-o", hobj]], verbose)
    tmp = LIB + ".tmp"
    _run([hipcc(), f"--offload-arch={ARCH}", "-shared", *[_object(s) for s in KERNEL_SRCS], hobj,
          "-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


def build_host_sanitized(out_dir: str, verbose: bool = False) -> str:
    """libdpmt with the host runtime under ASan + UBSan (every UB report
    fatal), linked with the kernels' objects of the in-tree build (compiled
    here if missing or older than their sources).  Returns the library path;
    it needs the ASan runtime preloaded (asan_runtime())."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    hdr = os.path.getmtime(os.path.join(CSRC, "dpmt_internal.h"))
    stale = [s for s in KERNEL_SRCS
             if not os.path.exists(_object(s)) or os.path.getmtime(_object(s)) < max(hdr, os.path.getmtime(s))]
    if stale:
        _compile_all([_kernel_cmd(s) for s in stale], verbose)
    kobjs = [_object(s) for s in KERNEL_SRCS]
    os.makedirs(out_dir, exist_ok=True)
    hobj = os.path.join(out_dir, "dpmt_host_san.o")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    _run([hipcc(), "--cuda-host-only", "-O1", "-g", *COMMON, *san, *_includes(), "-c", HOST_SRC,
          "-o", hobj], verbose)
    lib = os.path.join(out_dir, "libdpmt_san.so")
    _run([hipcc(), f"--offload-arch={ARCH}", "-shared", *san, *kobjs, hobj, "-o", lib], verbose)
    return lib


def asan_runtime() -> str:
    """Path of the compiler's shared ASan runtime (it carries the UBSan
    handlers too)."""
    res = subprocess.run([hipcc(), "--print-file-name=libclang_rt.asan-x86_64.so"],
                         capture_output=True, text=True)
    path = res.stdout.strip().splitlines()[-1] if res.stdout.strip() else ""
    if not os.path.isabs(path) or not os.path.exists(path):
        rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
        base = os.path.join(rocm, "llvm", "lib", "clang")
        for v in sorted(os.listdir(base)) if os.path.isdir(base) else []:
            cand = os.path.join(base, v, "lib", "linux", "libclang_rt.asan-x86_64.so")
            if os.path.exists(cand):
                return cand
        raise FileNotFoundError("libclang_rt.asan-x86_64.so not found")
    return path


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
    print(LIB)
