"""Build the qeh HIP library (libqeh.so) in-tree for gfx950 with hipcc.

Every call recompiles all sources (objects under _build/, one hipcc process
per source in parallel) and links paper_2104_10502_amd/libqeh.so.
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libqeh.so")
BUILD = os.path.join(ROOT, "_build")

HIP_SOURCES = ["fft_kernels.hip", "gemm_kernels.hip", "dav_kernels.hip", "beta_kernels.hip",
               "eigh_kernels.hip", "cg_kernels.hip"]
CPP_SOURCES = ["ctx.cpp", "davidson.cpp", "server.cpp", "beta.cpp", "cg.cpp"]

COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
          "-I" + os.path.join(ROOT, "include")]
# packed FP32 instructions are disabled for all device code
HIP_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-x", "hip"]


def _hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    is_hip = src.endswith(".hip")
    cmd = [_hipcc()] + COMMON + (HIP_FLAGS if is_hip else ["--offload-arch=gfx950", "-D__HIP_PLATFORM_AMD__"]) + \
        ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    if r.stderr.strip():
        warn = [ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if warn:
            sys.stderr.write("\n".join(warn) + "\n")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in HIP_SOURCES + CPP_SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = OUT + ".tmp"
    cmd = [_hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + \
        ["-L" + os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib"),
         "-lrocsolver", "-lrocblas", "-lamdhip64", "-Wl,-rpath," + os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"),
                                                       "lib")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


def build_host_sanitized(verbose: bool = False) -> str:
    """A copy of the library whose host C++ (validation, planning, maps,
    request copies, the Davidson state machine) is built with AddressSanitizer
    and UndefinedBehaviorSanitizer, linked with the regular device objects:
    _build/asan/libqeh_asan.so, for CPU tests of the host code.  The device
    code is not instrumented."""
    out_dir = os.path.join(BUILD, "asan")
    os.makedirs(out_dir, exist_ok=True)
    hip_objs = []
    for src in HIP_SOURCES:
        o = os.path.join(BUILD, src + ".o")
        if not os.path.exists(o):
            o = _compile(src)
        hip_objs.append(o)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-g"]

    def comp(src):
        obj = os.path.join(out_dir, src + ".o")
        cmd = [_hipcc()] + COMMON + ["--offload-arch=gfx950", "-D__HIP_PLATFORM_AMD__"] + san + \
            ["-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), r.stderr))
        return obj

    with cf.ThreadPoolExecutor(max_workers=len(CPP_SOURCES)) as ex:
        host_objs = list(ex.map(comp, CPP_SOURCES))
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    out = os.path.join(out_dir, "libqeh_asan.so")
    # linked by the LLVM driver (not hipcc) so that the shared sanitizer
    # runtime of the compiler that instrumented the objects is used
    cmd = [os.path.join(rocm, "llvm", "bin", "clang++"), "-shared", "-fPIC",
           "-fsanitize=address,undefined", "-shared-libsan", "-o", out] + host_objs + hip_objs + \
        ["-L" + os.path.join(rocm, "lib"), "-lrocsolver", "-lrocblas", "-lamdhip64",
         "-Wl,-rpath," + os.path.join(rocm, "lib")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), r.stderr))
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
