"""AddressSanitizer + UndefinedBehaviorSanitizer runs on the CPU (no GPU needed).

Builds the sanitizer variants of the oracle (oracle/build.py build_sanitized) and of the library's
host-side sources (paper_2606_26297_amd/build.py build_sanitized: validation, planning, allocation
strategies and search driver instrumented, device objects of the regular build linked in), then runs
tests/sanitize_driver.py on each in a fresh process with the LLVM sanitizer runtime preloaded.  Any
sanitizer report aborts that process; the test also fails on a report that did not abort.
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "tests", "sanitize_driver.py")


def runtime():
    found = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not found:
        pytest.skip("the LLVM AddressSanitizer runtime is not installed")
    return found[-1]


def run_driver(args):
    env = dict(os.environ)
    # the sanitizer runtime must come first among preloaded libraries; anything already preloaded stays
    env["LD_PRELOAD"] = ":".join([runtime()] + ([os.environ["LD_PRELOAD"]] if os.environ.get("LD_PRELOAD") else []))
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["HIP_VISIBLE_DEVICES"] = ""  # host paths only, also on a machine with a GPU
    r = subprocess.run([sys.executable, DRIVER, *args], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    report = "ERROR: AddressSanitizer" in r.stderr or "runtime error:" in r.stderr
    assert r.returncode == 0 and not report, r.stdout[-2000:] + r.stderr[-6000:]
    return r.stdout


def test_oracle_under_sanitizers():
    out = run_driver(["oracle"])
    assert "sanitized build equals the regular build" in out


def test_library_host_code_under_sanitizers():
    sys.path.insert(0, ROOT)
    from paper_2606_26297_amd import build as B

    lib = B.build_sanitized()
    out = run_driver(["library", lib])
    assert "ran clean" in out
