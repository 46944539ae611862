"""TEST INFRASTRUCTURE -- the oracle of the gate-level distributed circuit with explicit TeleGate
remote CNOTs (distributed circuit construction section).

Only tests may import this module; the product never does.  A plain numpy statevector of n data
qubits plus two communication qubits (qubit n on the control's QPU, n + 1 on the target's), complex128:

* per layer: the phase of every term local to a QPU (C minus the cross-QPU couplings, eq. (16));
  then each cross-QPU coupling b z_i z_j (i < j, row-major) as single-qubit phases
  diag(1, e^{-i gamma b / 2}) on i and j and the parity phase e^{+i gamma b (z_i xor z_j) / 2}, i.e.
  CNOT(i -> j), diag(1, e^{+i gamma b / 2}) on j, CNOT(i -> j), both CNOTs remote; then RX(2 beta)
  on every data qubit (eq. (12)-(13));
* a remote CNOT: the communication pair is entangled (H on qubit n, CNOT n -> n + 1), the control is
  coupled to qubit n, which is measured (outcome m1), qubit n + 1 is coupled to the target, turned by
  H and measured (m2); X^m1 on the target and Z^m2 on the control correct the data qubits, and both
  communication qubits are reset to |0>; what remains is the global phase (-1)^(m1 m2), which the
  simulation removes so that trajectories compare with the exact state;
* a measurement gives 1 when the caller's uniform is below the probability of 1, and keeps the
  renormalised branch.

Each cross-QPU term takes two remote CNOTs, so a layer takes 2 x cross of them (the estimate of the
allocation section).
"""
from __future__ import annotations

import numpy as np


class Circuit:
    def __init__(self, n):
        self.n = n
        self.nq = n + 2
        self.psi = np.zeros(1 << self.nq, dtype=np.complex128)
        self.psi[: 1 << n] = 1.0 / np.sqrt(1 << n)
        self.outcomes = []

    def _bit(self, q):
        return (np.arange(self.psi.size, dtype=np.int64) >> q) & 1

    def phase(self, q, phi):
        self.psi[self._bit(q) == 1] *= np.exp(1j * phi)

    def cnot(self, c, t):
        z = np.arange(self.psi.size, dtype=np.int64)
        sel = (((z >> c) & 1) == 1) & (((z >> t) & 1) == 0)
        a = self.psi[z[sel]].copy()
        self.psi[z[sel]] = self.psi[z[sel] | (1 << t)]
        self.psi[z[sel] | (1 << t)] = a

    def one(self, q, M):
        z = np.arange(self.psi.size, dtype=np.int64)
        lo = z[((z >> q) & 1) == 0]
        a, b = self.psi[lo].copy(), self.psi[lo | (1 << q)].copy()
        self.psi[lo] = M[0, 0] * a + M[0, 1] * b
        self.psi[lo | (1 << q)] = M[1, 0] * a + M[1, 1] * b

    def h(self, q):
        self.one(q, np.array([[1, 1], [1, -1]]) / np.sqrt(2.0))

    def x(self, q):
        self.one(q, np.array([[0, 1], [1, 0]], dtype=complex))

    def z(self, q):
        self.one(q, np.array([[1, 0], [0, -1]], dtype=complex))

    def measure(self, q, u):
        bit = self._bit(q)
        p1 = float(np.sum(np.abs(self.psi[bit == 1]) ** 2))
        m = 1 if u < p1 else 0
        keep = bit == m
        self.psi[~keep] = 0.0
        self.psi[keep] /= np.sqrt(p1 if m else 1.0 - p1)
        self.outcomes.append(m)
        return m, p1

    def remote_cnot(self, c, t, u1, u2):
        a, b = self.n, self.n + 1
        self.h(a)
        self.cnot(a, b)
        self.cnot(c, a)
        m1, _ = self.measure(a, u1)
        self.cnot(b, t)
        self.h(b)
        m2, _ = self.measure(b, u2)
        if m1:
            self.x(t)
        if m2:
            self.z(c)
        if m1:
            self.x(a)
        if m2:
            self.x(b)
        if m1 and m2:  # the protocol leaves the global phase (-1)^(m1 m2); removed to compare states
            self.psi *= -1.0

    def data_state(self):
        return self.psi[: 1 << self.n].copy()


def cross_terms_list(b, q):
    """Cross-QPU couplings (i, j, b_ij), i < j, row-major."""
    n = b.shape[0]
    return [(i, j, b[i, j]) for i in range(n) for j in range(i + 1, n) if b[i, j] != 0.0 and q[i] != q[j]]


def trajectory(local_diag, b, q, x, uniforms):
    """Final data state and outcomes.  local_diag: the cost of the QPU-local terms for every z
    (C minus the cross couplings); b: canonical couplings (upper triangle); q: QPU of each variable;
    x: interleaved angles; uniforms: two per remote CNOT, in circuit order."""
    n = b.shape[0]
    p = len(x) // 2
    cross = cross_terms_list(b, q)
    circ = Circuit(n)
    u = list(np.asarray(uniforms, dtype=np.float64).ravel())
    pos = 0
    full_local = np.tile(np.asarray(local_diag, dtype=np.float64), 4)  # the communication bits do not enter
    for k in range(p):
        g, be = x[2 * k], x[2 * k + 1]
        circ.psi *= np.exp(-1j * g * full_local)
        for i, j, bij in cross:
            circ.phase(i, -g * bij / 2.0)
            circ.phase(j, -g * bij / 2.0)
            circ.remote_cnot(i, j, u[pos], u[pos + 1])
            circ.phase(j, g * bij / 2.0)
            circ.remote_cnot(i, j, u[pos + 2], u[pos + 3])
            pos += 4
        rx = np.array([[np.cos(be), -1j * np.sin(be)], [-1j * np.sin(be), np.cos(be)]])
        for qq in range(n):
            circ.one(qq, rx)
    return circ.data_state(), circ.outcomes, 2 * len(cross) * p
