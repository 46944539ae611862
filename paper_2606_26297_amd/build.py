"""Build libqaoa_qubo.so (the HIP kernels and the C ABI) for gfx950 with hipcc.

Usage: python -m paper_2606_26297_amd.build [--verbose] [--resource-usage]
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libqaoa_qubo.so")
BUILD_DIR = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# host-only sources (no kernels): plain C++ against the HIP runtime headers, no device code objects
CXX = os.environ.get("QQ_HOST_CXX", "/opt/rocm/llvm/bin/clang++")
HOST = ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]
ARCH = "gfx950"

HIP_SOURCES = ["qq_kernels.hip", "qq_fast.hip", "qq_many.hip", "qq_optim.hip", "qq_plain.hip", "qq_sample.hip",
               "qq_telegate.hip", "qq_static.hip"]
CPP_SOURCES = ["qq_api.cpp", "qq_driver.cpp", "qq_alloc.cpp"]

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function"]
# Device code: gfx950 only; packed FP32 instructions disabled.
DEVICE = ["-x", "hip", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-ffp-contract=fast"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}")
    return r.stdout + r.stderr


def build(verbose: bool = False, resource_usage: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    jobs = []
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD_DIR, src + ".o")
        extra = ["-Rpass-analysis=kernel-resource-usage"] if resource_usage else []
        jobs.append([HIPCC, *COMMON, *DEVICE, *extra, "-c", os.path.join(CSRC, src), "-o", obj])
    for src in CPP_SOURCES:
        obj = os.path.join(BUILD_DIR, src + ".o")
        jobs.append([CXX, *COMMON, *HOST, "-c", os.path.join(CSRC, src), "-o", obj])
    with cf.ThreadPoolExecutor(max_workers=min(6, len(jobs))) as ex:
        outs = list(ex.map(lambda c: _run(c, verbose), jobs))
    if resource_usage:
        for o in outs:
            sys.stdout.write(o)
    objs = [os.path.join(BUILD_DIR, s + ".o") for s in HIP_SOURCES + CPP_SOURCES]
    tmp = LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs], verbose)
    os.replace(tmp, LIB)
    return LIB


# AddressSanitizer + UndefinedBehaviorSanitizer build of the host-side sources (validation, planning,
# allocation strategies, search driver) for CPU tests: they are compiled again with the sanitizers
# and linked with the device objects of the regular build into a separate library.  The sanitizer
# runtime is not linked in; the test that loads this library preloads it.
SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
SAN_DIR = os.path.join(BUILD_DIR, "san")
SAN_LIB = os.path.join(SAN_DIR, "libqaoa_qubo_san.so")


def build_sanitized(verbose: bool = False) -> str:
    dev_objs = [os.path.join(BUILD_DIR, s + ".o") for s in HIP_SOURCES]
    if not all(os.path.exists(o) for o in dev_objs):
        build(verbose)
    os.makedirs(SAN_DIR, exist_ok=True)
    objs = []
    for src in CPP_SOURCES:
        obj = os.path.join(SAN_DIR, src + ".o")
        _run([CXX, "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", *SAN_FLAGS, *HOST, "-c",
              os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    tmp = SAN_LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, *dev_objs], verbose)
    os.replace(tmp, SAN_LIB)
    return SAN_LIB


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        print(build_sanitized(verbose="--verbose" in sys.argv))
    else:
        print(build(verbose="--verbose" in sys.argv, resource_usage="--resource-usage" in sys.argv))
