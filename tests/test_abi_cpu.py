"""Host-side checks of the C ABI that need no GPU: the library loads, exports every
symbol the header declares, and rejects invalid input before any device work."""
import ctypes
import subprocess

import numpy as np
import pytest

from paper_2606_26297_amd import native as N


@pytest.fixture(scope="module")
def L():
    return N.lib()


def test_header_declares_the_boundary():
    syms = N.header_symbols()
    for name in ["qq_problem_create", "qq_evaluate", "qq_state", "qq_topk", "qq_set_allocation",
                 "qq_cost_diagonal", "qq_workspace_size", "qq_evaluate_plain", "qq_last_error"]:
        assert name in syms
    assert set(syms) == set(N.SIGNATURES), "binding and header disagree"


def test_library_exports_every_header_symbol(L):
    out = subprocess.run(["nm", "-D", "--defined-only", N.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = [s for s in N.header_symbols() if s not in exported]
    assert not missing, missing
    for s in N.header_symbols():
        assert hasattr(L, s)
    assert N.qq_abi_version() == 1


def test_device_count_without_gpu_is_not_an_error(L):
    assert N.qq_device_count() >= 0


@pytest.mark.parametrize("n", [0, -3, N.QQ_MAX_N + 1, 40])
def test_create_rejects_bad_n(L, n):
    H = np.zeros((max(n, 1), max(n, 1)))
    with pytest.raises(N.QQError) as ei:
        N.qq_problem_create(n, H)
    assert ei.value.status == N.QQ_E_INVALID
    assert "n =" in N.qq_last_error()


def test_create_rejects_non_finite(L):
    H = np.eye(4)
    H[1, 2] = np.nan
    with pytest.raises(N.QQError) as ei:
        N.qq_problem_create(4, H)
    assert ei.value.status == N.QQ_E_INVALID and "H[1][2]" in str(ei.value)
    f = np.array([0.0, np.inf, 0.0, 0.0])
    with pytest.raises(N.QQError) as ei:
        N.qq_problem_create(4, np.eye(4), f)
    assert ei.value.status == N.QQ_E_INVALID and "f[1]" in str(ei.value)
    with pytest.raises(N.QQError) as ei:
        N.qq_problem_create(4, np.eye(4), None, float("nan"))
    assert ei.value.status == N.QQ_E_INVALID


def test_null_arguments_are_rejected(L):
    out = ctypes.c_void_p()
    assert L.qq_problem_create(3, None, None, 0.0, 0, None, ctypes.byref(out)) == N.QQ_E_INVALID
    H = np.eye(3)
    assert L.qq_problem_create(3, H.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None, 0.0, 0, None,
                               None) == N.QQ_E_INVALID
    info = N.QQInfo()
    assert L.qq_problem_info(None, ctypes.byref(info)) == N.QQ_E_INVALID
    s = ctypes.c_size_t(0)
    assert L.qq_workspace_size(None, 1, 1, 1, ctypes.byref(s)) == N.QQ_E_INVALID
    assert L.qq_evaluate(None, 1, 1, None, 1, None, 0, None, None, None) == N.QQ_E_INVALID
    assert L.qq_set_allocation(None, 2, None, None, None, None) == N.QQ_E_INVALID
    assert N.qq_last_error()


def test_guarded_calls_reject_bad_arguments_before_device_work(L):
    dp = ctypes.POINTER(ctypes.c_double)
    x = np.array([0.1, 0.2])
    e = np.zeros(1)
    assert L.qq_evaluate_guarded(None, 1, 1, x.ctypes.data_as(dp), N.QQ_ENERGY | N.QQ_GRAD, 1e-5, None,
                                 e.ctypes.data_as(dp), None, None, None) == N.QQ_E_INVALID
    assert "NULL" in N.qq_last_error()
    assert L.qq_evaluate_many_guarded(0, None, None, None, None, N.QQ_ENERGY, None, 1e-5, None, None, None, None,
                                      None) == N.QQ_E_INVALID


def test_guard_constants_match_the_header():
    import re

    text = open(N.HEADER).read()
    assert float(re.search(r"#define QQ_GUARD_REL (\S+)", text).group(1)) == N.QQ_GUARD_REL
    assert float(re.search(r"#define QQ_GUARD_K (\S+)", text).group(1)) == N.QQ_GUARD_K
