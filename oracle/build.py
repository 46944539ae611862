"""Compile the C oracle (test infrastructure) into oracle/liboracle.so with gcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "qaoa_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


# AddressSanitizer + UndefinedBehaviorSanitizer build of the same source (CPU tests only), with the
# LLVM C compiler of the toolchain so that it shares one sanitizer runtime with the host-library
# build of paper_2606_26297_amd/build.py.
CLANG = os.environ.get("QQ_SAN_CC", "/opt/rocm/llvm/bin/clang")
SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
SAN_LIB = os.path.join(HERE, "liboracle_san.so")


def build_sanitized() -> str:
    tmp = SAN_LIB + ".tmp"
    cmd = [CLANG, "-std=c99", "-ffp-contract=off", "-fPIC", "-shared", "-Wall", *SAN_FLAGS, SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, SAN_LIB)
    return SAN_LIB


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        print(build_sanitized())
    else:
        print(build(force="--lazy" not in sys.argv))
