"""Runs the AddressSanitizer / UndefinedBehaviorSanitizer builds of the oracle and of the library's
host-side code on the CPU (started by test_sanitizers_cpu.py in a subprocess with the sanitizer
runtime preloaded; not collected by pytest itself).

  * oracle (liboracle_san.so): canonical form, integer and real diagonals, phase and mixer, states,
    expectation and adjoint gradient on small n, each compared with the regular oracle build (the
    diagonals bit for bit, the rest to the last places that two compilers may round differently);
  * library (libqaoa_qubo_san.so, host code instrumented): every validation path that runs before
    device work (sizes, NULL pointers, non-finite values, flags, allocations, guarded, static and
    many-problem calls), and the host-only allocation strategies on random problems.
Exits non-zero on the first mismatch; a sanitizer finding aborts the process.
"""
from __future__ import annotations

import ctypes
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def oracle_checks():
    from oracle import build as ob
    from oracle import oracle as O

    rng = np.random.default_rng(11)
    cases = []
    for n in (1, 2, 3, 5, 6):
        H = rng.integers(-5, 6, size=(n, n)).astype(float)
        f = rng.integers(-3, 4, size=n).astype(float)
        x = rng.uniform(0, np.pi, size=4)
        cases.append((H, f, 2.0, x))
        Hr = rng.normal(size=(n, n))
        cases.append((Hr, rng.normal(size=n), -0.5, rng.uniform(0, np.pi, size=6)))

    def run_all():
        out = []
        for H, f, c0, x in cases:
            d = O.cost_diagonal(H, f, c0)
            psi = O.qaoa_state(d, x)
            e, g = O.gradient(d, x)
            ell, b = O.canonicalise(H, f)
            n = H.shape[0]
            M = min(2, n)
            parts = O.partitioned_diagonals(H, f, c0, np.arange(n) % M, M)
            out.append((d.copy(), psi.copy(), e, g.copy(), ell.copy(), b.copy(),
                        [np.array(v, copy=True) for v in parts[:1]]))
        return out

    ref = run_all()
    O._LIB = None
    san = ctypes.CDLL(ob.build_sanitized())
    orig_build = ob.build
    ob.build = lambda force=False: ob.SAN_LIB
    try:
        got = run_all()
    finally:
        ob.build = orig_build
    assert O._lib()._name == ob.SAN_LIB and san is not None
    # the diagonals and the canonical form are sums in a fixed order (bit-identical across compilers);
    # states, energies and gradients go through libm and complex arithmetic that two compilers may
    # round differently in the last place
    for a, b in zip(ref, got):
        d0, psi0, e0, g0, ell0, b0, parts0 = a
        d1, psi1, e1, g1, ell1, b1, parts1 = b
        assert np.array_equal(d0, d1) and np.array_equal(ell0, ell1) and np.array_equal(b0, b1)
        assert all(np.array_equal(u, v) for u, v in zip(parts0, parts1))
        assert np.max(np.abs(psi0 - psi1)) <= 1e-13
        assert abs(e0 - e1) <= 1e-12 * max(1.0, abs(e0)) and np.max(np.abs(g0 - g1)) <= 1e-12 * max(1.0, np.max(np.abs(g0)))
    print("oracle: sanitized build equals the regular build on", len(cases), "problems", flush=True)


def library_checks(path):
    from paper_2606_26297_amd import native as N

    L = ctypes.CDLL(path)
    for name, (args, res) in N.SIGNATURES.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    N._LIB = L  # no torch import: host paths only
    dp = ctypes.POINTER(ctypes.c_double)

    def status(fn):
        try:
            fn()
        except N.QQError as e:
            return e.status
        return N.QQ_OK

    assert N.qq_abi_version() == 1
    assert N.qq_device_count() >= 0
    H = np.eye(4)
    for n in (0, -1, N.QQ_MAX_N + 1):
        assert status(lambda: N.qq_problem_create(n, np.zeros((max(n, 1), max(n, 1))))) == N.QQ_E_INVALID
    Hn = H.copy()
    Hn[2, 3] = np.nan
    assert status(lambda: N.qq_problem_create(4, Hn)) == N.QQ_E_INVALID
    assert status(lambda: N.qq_problem_create(4, H, np.array([0, np.inf, 0, 0.0]))) == N.QQ_E_INVALID
    assert status(lambda: N.qq_problem_create(4, H, None, float("nan"))) == N.QQ_E_INVALID
    out = ctypes.c_void_p()
    assert L.qq_problem_create(3, None, None, 0.0, 0, None, ctypes.byref(out)) == N.QQ_E_INVALID
    info = N.QQInfo()
    assert L.qq_problem_info(None, ctypes.byref(info)) == N.QQ_E_INVALID
    s = ctypes.c_size_t(0)
    assert L.qq_workspace_size(None, 1, 1, 1, ctypes.byref(s)) == N.QQ_E_INVALID
    x = np.array([0.1, 0.2])
    e = np.zeros(1)
    assert L.qq_evaluate(None, 1, 1, x.ctypes.data_as(dp), 1, None, 0, None, e.ctypes.data_as(dp), None) \
        == N.QQ_E_INVALID
    assert L.qq_evaluate_static(None, 1, 1, x.ctypes.data_as(dp), 1, None, e.ctypes.data_as(dp), None) \
        == N.QQ_E_INVALID
    assert L.qq_evaluate_guarded(None, 1, 1, x.ctypes.data_as(dp), 3, 1e-5, None, e.ctypes.data_as(dp), None, None,
                                 None) == N.QQ_E_INVALID
    assert L.qq_evaluate_many(0, None, None, None, None, 1, None, None, 0, None, None, None) == N.QQ_E_INVALID
    assert L.qq_evaluate_many_guarded(0, None, None, None, None, 1, None, 1e-5, None, None, None, None, None) \
        == N.QQ_E_INVALID
    assert L.qq_set_allocation(None, 2, None, None, None, None) == N.QQ_E_INVALID
    assert N.qq_last_error()
    # host-only allocation strategies on random problems
    rng = np.random.default_rng(12)
    for n in (2, 5, 9, 16, 24):
        for M in sorted({1, 2, min(n, 3), min(n, 5)}):
            caps = N.qq_balanced_capacities(n, M)
            assert caps.sum() == n and caps.max() - caps.min() <= 1
            Hq = rng.normal(size=(n, n)) * (rng.random((n, n)) < 0.4)
            for strat in (N.QQ_ALLOC_CONTIGUOUS, N.QQ_ALLOC_GRAPH):
                q, cross = N.qq_allocation(Hq, M, caps, strat)
                assert np.all((q >= 0) & (q < M)) and cross >= 0
                assert np.array_equal(np.bincount(q, minlength=M), caps)
            qs, cr, rem, best = N.qq_allocation_candidates(Hq, M, 3, caps)
            assert np.all(rem == 2 * 3 * cr) and 0 <= best < len(cr)
    assert status(lambda: N.qq_balanced_capacities(3, 0)) == N.QQ_E_INVALID
    assert status(lambda: N.qq_allocation(np.eye(3), 4, [1, 1, 1, 1])) != N.QQ_OK
    print("library: validation paths and allocation strategies ran clean", flush=True)


if __name__ == "__main__":
    assert hasattr(ctypes.CDLL(None), "__asan_report_load8"), "the AddressSanitizer runtime is not loaded"
    # usage: sanitize_driver.py oracle | sanitize_driver.py library <path of libqaoa_qubo_san.so>
    if sys.argv[1] == "oracle":
        oracle_checks()
    else:
        library_checks(sys.argv[2])
