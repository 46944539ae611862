"""TEST INFRASTRUCTURE -- the FP64 CPU oracle for the exact QAOA-for-QUBO path.

Only tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import this module.  The product (the HIP library and its binding) never
does.  The heavy loops live in ``qaoa_oracle.c`` (plain C, single thread,
FP64); this file adds the small host-side pieces in numpy, each following the
passage of the paper cited on it:

* canonical form and integrality (eq. (3)-(6));
* Ising / Pauli coefficients alpha, h, J of eq. (9), which the paper does not
  write out -- derived here by substituting z_i = (1 - Z_i)/2 (eq. (7)) into
  eq. (8);
* probabilities, top-k and best bitstrings (decoding and metrics section):
  ties go to the lowest basis index;
* local / cross-QPU split of the couplings (eq. (16)), cross counts and the
  remote-CNOT estimate 2 * cross * p of the allocation section;
* central finite differences, used only to pin the adjoint gradient.

Bit convention: variable z_i (i = 1..n) is bit (i-1) of the basis index;
printed bitstrings are z_1 z_2 ... z_n (the reversal of the little-endian
display described in the decoding section).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int64)


def _lib():
    global _LIB
    if _LIB is None:
        from oracle import build as _build  # local build helper (gcc)

        path = _build.build(force=False)
        lib = ctypes.CDLL(path)
        lib.orc_canonicalise.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp]
        lib.orc_cost_diag_int.argtypes = [ctypes.c_int, _ip, _ip, ctypes.c_int64, _ip]
        lib.orc_cost_diag_real.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_double, _dp]
        lib.orc_apply_phase.argtypes = [ctypes.c_int, _dp, ctypes.c_double, ctypes.c_int, _dp]
        lib.orc_apply_mixer.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int, _dp]
        lib.orc_qaoa_state.argtypes = [ctypes.c_int, _dp, ctypes.c_int, _dp, _dp]
        lib.orc_qaoa_state_multi.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _dp, _dp]
        lib.orc_expectation.argtypes = [ctypes.c_int, _dp, _dp]
        lib.orc_expectation.restype = ctypes.c_double
        lib.orc_adjoint_gradient.argtypes = [ctypes.c_int, _dp, ctypes.c_int, _dp, _dp]
        lib.orc_adjoint_gradient.restype = ctypes.c_double
        _LIB = lib
    return _LIB


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


# --- canonical form (eq. (3)-(6)) ----------------------------------------------------------

def canonicalise(H, f=None):
    """Return (l, b): l_i = f_i + H_ii, b_ij = H_ij + H_ji for i < j (b as n x n, strict upper)."""
    H = np.ascontiguousarray(H, dtype=np.float64)
    n = H.shape[0]
    f = np.zeros(n) if f is None else np.ascontiguousarray(f, dtype=np.float64)
    ell = np.zeros(n)
    b = np.zeros((n, n))
    _lib().orc_canonicalise(n, _d(H), _d(f), _d(ell), _d(b))
    return ell, b


INT_BOUND = 2**31


def is_integer_problem(H, f=None, c0=0.0) -> bool:
    """Integral H, f and c0 whose canonical magnitudes sum below 2^31 (so every C(z) fits int32)."""
    H = np.asarray(H, dtype=np.float64)
    f = np.zeros(H.shape[0]) if f is None else np.asarray(f, dtype=np.float64)
    vals = np.concatenate([H.ravel(), f.ravel(), [float(c0)]])
    if not np.all(np.isfinite(vals)) or not np.all(vals == np.round(vals)):
        return False
    ell, b = canonicalise(H, f)
    return float(np.abs(ell).sum() + np.abs(np.triu(b, 1)).sum() + abs(float(c0))) < INT_BOUND


def cost_diagonal(H, f=None, c0=0.0):
    """C(z) for every basis index z (eq. (6)); int64 for integer problems, else float64."""
    ell, b = canonicalise(H, f)
    n = ell.shape[0]
    if is_integer_problem(H, f, c0):
        e = np.ascontiguousarray(np.round(ell).astype(np.int64))
        bb = np.ascontiguousarray(np.round(b).astype(np.int64))
        out = np.empty(1 << n, dtype=np.int64)
        _lib().orc_cost_diag_int(n, _i(e), _i(bb), int(round(c0)), _i(out))
        return out
    return cost_diagonal_real(ell, b, c0)


def cost_diagonal_real(ell, b, c0):
    """FP64 diagonal of canonical coefficients in the canonical summation order."""
    ell = np.ascontiguousarray(ell, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    n = ell.shape[0]
    out = np.empty(1 << n, dtype=np.float64)
    _lib().orc_cost_diag_real(n, _d(ell), _d(b), float(c0), _d(out))
    return out


def cost_at_real(ell, b, c0, z):
    """C(z) of eq. (6) for one basis index z, real coefficients, FP64 in the canonical order: c0,
    then l_i over the set bits in ascending i, then b_ij over the set pairs row by row (the order of
    cost_diagonal_real, one index at a time, so full-size diagonals can be checked at sampled z)."""
    n = len(ell)
    acc = float(c0)
    for i in range(n):
        if (z >> i) & 1:
            acc += float(ell[i])
    for i in range(n):
        if (z >> i) & 1:
            for j in range(i + 1, n):
                if (z >> j) & 1:
                    acc += float(b[i][j])
    return acc


# --- Ising / Pauli form (eq. (7)-(9)) -------------------------------------------------------

def ising_coefficients(ell, b, c0):
    """alpha, h, J with H_C = alpha I + sum h_i Z_i + sum_{i<j} J_ij Z_i Z_j.

    From z_i = (1 - Z_i)/2:  l_i z_i -> l_i/2 - (l_i/2) Z_i and
    b_ij z_i z_j -> (b_ij/4)(1 - Z_i - Z_j + Z_i Z_j), so
    alpha = c0 + sum l/2 + sum b/4,  h_i = -l_i/2 - sum_{j != i} b_{ij}/4,  J_ij = b_ij/4.
    sigma_C = sqrt(sum h^2 + sum J^2) is the standard deviation of C over uniform z.
    """
    ell = np.asarray(ell, dtype=np.float64)
    bu = np.triu(np.asarray(b, dtype=np.float64), 1)
    bs = bu + bu.T
    alpha = float(c0) + ell.sum() / 2.0 + bu.sum() / 4.0
    h = -ell / 2.0 - bs.sum(axis=1) / 4.0
    J = bu / 4.0
    sigma = float(np.sqrt((h**2).sum() + (J**2).sum()))
    return alpha, h, J, sigma


# --- statevector (eq. (10)-(13)) ------------------------------------------------------------

def _as_f64_diag(diag):
    return np.ascontiguousarray(np.asarray(diag).astype(np.float64))


def qaoa_state(diag, x):
    """|gamma, beta> of eq. (11) as complex128[2^n]; x = [g1, b1, ..., gp, bp]."""
    d = _as_f64_diag(diag)
    n = int(d.shape[0]).bit_length() - 1
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    p = x.shape[0] // 2
    psi = np.empty(1 << n, dtype=np.complex128)
    _lib().orc_qaoa_state(n, _d(d), p, _d(x), psi.ctypes.data_as(_dp))
    return psi


def qaoa_state_multi(diags, x):
    """State whose every cost layer applies exp(-i gamma C_d) for each diagonal d in order."""
    D = np.ascontiguousarray(np.stack([_as_f64_diag(d) for d in diags]))
    n = int(D.shape[1]).bit_length() - 1
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    psi = np.empty(1 << n, dtype=np.complex128)
    _lib().orc_qaoa_state_multi(n, D.shape[0], _d(D), x.shape[0] // 2, _d(x), psi.ctypes.data_as(_dp))
    return psi


def apply_phase(diag, gamma, psi, sign=+1):
    d = _as_f64_diag(diag)
    out = np.ascontiguousarray(psi, dtype=np.complex128).copy()
    n = int(d.shape[0]).bit_length() - 1
    _lib().orc_apply_phase(n, _d(d), float(gamma), int(sign), out.ctypes.data_as(_dp))
    return out


def apply_mixer(beta, psi, sign=+1):
    out = np.ascontiguousarray(psi, dtype=np.complex128).copy()
    n = int(out.shape[0]).bit_length() - 1
    _lib().orc_apply_mixer(n, float(beta), int(sign), out.ctypes.data_as(_dp))
    return out


def expectation(diag, psi):
    """eq. (15): sum_z |psi(z)|^2 C(z)."""
    d = _as_f64_diag(diag)
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    n = int(d.shape[0]).bit_length() - 1
    return float(_lib().orc_expectation(n, _d(d), psi.ctypes.data_as(_dp)))


def energy(diag, x):
    """J(x) of eq. (17), exactly (no shot sampling)."""
    return expectation(diag, qaoa_state(diag, x))


def gradient(diag, x):
    """(E, dE/dx) by the adjoint sweep; dE/dx interleaved like x."""
    d = _as_f64_diag(diag)
    n = int(d.shape[0]).bit_length() - 1
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    g = np.empty_like(x)
    e = _lib().orc_adjoint_gradient(n, _d(d), x.shape[0] // 2, _d(x), _d(g))
    return float(e), g


def fd_gradient(diag, x, h=1e-6):
    """Central finite differences (E(x + h e_j) - E(x - h e_j)) / 2h, FP64."""
    x = np.asarray(x, dtype=np.float64).ravel()
    g = np.empty_like(x)
    for j in range(x.shape[0]):
        xp = x.copy()
        xm = x.copy()
        xp[j] += h
        xm[j] -= h
        g[j] = (energy(diag, xp) - energy(diag, xm)) / (2.0 * h)
    return g


# --- distribution metrics (decoding / metrics section) ---------------------------------------

def probabilities(psi):
    psi = np.asarray(psi)
    return psi.real.astype(np.float64) ** 2 + psi.imag.astype(np.float64) ** 2


def topk(P, k):
    """Indices of the k largest probabilities, ordered by (-P, index)."""
    P = np.asarray(P, dtype=np.float64)
    idx = np.arange(P.shape[0])
    order = np.lexsort((idx, -P))
    return order[:k]


def argmin_cost(diag):
    """Lowest-index minimiser of C (the brute-force optimum of the classical reference mode)."""
    d = np.asarray(diag)
    return int(np.flatnonzero(d == d.min())[0])


def bitstring(index: int, n: int) -> str:
    """Logical bitstring z_1 ... z_n of a basis index (z_i = bit i-1)."""
    return "".join("1" if (index >> i) & 1 else "0" for i in range(n))


def index_from_display(display: str) -> int:
    """Basis index from a little-endian display string b_{n-1} ... b_0."""
    return int(display, 2)


# --- allocation (eq. (16) and the allocation section) ---------------------------------------

def balanced_capacities(n: int, M: int):
    """Capacities as even as possible: c_m = floor(n/M) + [m < n mod M]."""
    return [n // M + (1 if m < n % M else 0) for m in range(M)]


def validate_allocation(q, M, capacities=None):
    """Each variable on exactly one QPU in [0, M), no capacity exceeded, every QPU used."""
    q = np.asarray(q)
    if q.ndim != 1 or np.any(q < 0) or np.any(q >= M):
        return False
    counts = np.bincount(q, minlength=M)
    if np.any(counts == 0):
        return False
    if capacities is not None and np.any(counts > np.asarray(capacities)):
        return False
    return True


def cross_terms(b, q):
    """Number of nonzero couplings b_ij (i < j) with q(i) != q(j)  (eq. (16))."""
    bu = np.triu(np.asarray(b), 1)
    q = np.asarray(q)
    i, j = np.nonzero(bu)
    return int(np.count_nonzero(q[i] != q[j]))


def remote_cx_estimate(cross: int, p: int) -> int:
    """Two remote CNOTs per cross-QPU term per layer."""
    return 2 * int(cross) * int(p)


def split_by_allocation(ell, b, c0, q, M):
    """Canonical coefficients of the per-QPU local parts and of the cross part (eq. (16)).

    Part m (m = 0..M-1) keeps l_i for q(i) = m and b_ij with q(i) = q(j) = m;
    the constant c0 goes to part 0.  The cross part keeps b_ij with q(i) != q(j).
    Returns a list of M + 1 triples (l, b, c0).
    """
    ell = np.asarray(ell, dtype=np.float64)
    bu = np.triu(np.asarray(b, dtype=np.float64), 1)
    q = np.asarray(q)
    same = q[:, None] == q[None, :]
    parts = []
    for m in range(M):
        on = q == m
        lm = np.where(on, ell, 0.0)
        bm = np.where(same & on[:, None], bu, 0.0)
        parts.append((lm, bm, float(c0) if m == 0 else 0.0))
    parts.append((np.zeros_like(ell), np.where(~same, bu, 0.0), 0.0))
    return parts


def partitioned_diagonals(H, f, c0, q, M):
    """Full-length diagonals of every part of split_by_allocation, in application order."""
    ell, b = canonicalise(H, f)
    return [cost_diagonal_real(lm, bm, cm) for (lm, bm, cm) in split_by_allocation(ell, b, c0, q, M)]
