"""Pins of the oracle's TeleGate circuit (CPU only).

* One remote CNOT on a random state of four data qubits, for each of the four outcome pairs (forced
  through the uniforms: every measurement of the protocol has probability 1/2): the data state
  afterwards equals the CNOT matrix applied to the state before, the communication qubits are back
  in |00>, and each measurement's probability of 1 is 1/2.
* Whole trajectories (random outcomes) of the distributed circuit equal the exact QAOA state of the
  monolithic oracle (eq. (11)) to 1e-12, global phase included, for several allocations; the number
  of remote CNOTs is 2 x cross x p.
"""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import telegate as T
from paper_2606_26297_amd import workloads as W


def cnot_reference(psi, c, t):
    out = psi.copy()
    for z in range(psi.size):
        if (z >> c) & 1:
            out[z ^ (1 << t)] = psi[z]
    return out


@pytest.mark.parametrize("c,t", [(0, 3), (2, 1)])
@pytest.mark.parametrize("u1,u2", [(0.25, 0.25), (0.25, 0.75), (0.75, 0.25), (0.75, 0.75)])
def test_one_remote_cnot_all_outcomes(c, t, u1, u2):
    rng = np.random.default_rng(7 + 3 * c + t)
    psi = rng.normal(size=16) + 1j * rng.normal(size=16)
    psi /= np.linalg.norm(psi)
    circ = T.Circuit(4)
    circ.psi[:] = 0.0
    circ.psi[:16] = psi
    probs = []
    orig = circ.measure

    def measure(q, u):
        m, p1 = orig(q, u)
        probs.append(p1)
        return m, p1

    circ.measure = measure
    circ.remote_cnot(c, t, u1, u2)
    assert circ.outcomes == [int(u1 < 0.5), int(u2 < 0.5)]
    assert np.allclose(probs, 0.5, atol=1e-14)
    assert np.linalg.norm(circ.psi[16:]) <= 1e-14
    assert np.linalg.norm(circ.data_state() - cnot_reference(psi, c, t)) <= 1e-13


@pytest.mark.parametrize("n,M,seed", [(5, 2, 1), (6, 3, 2), (7, 2, 3)])
def test_trajectory_equals_exact_state(n, M, seed):
    inst = W.dense_gaussian_upper(n, 90 + seed)
    caps = O.balanced_capacities(n, M)
    q = W.contiguous_allocation(n, caps)
    parts = O.partitioned_diagonals(inst.H, inst.f, inst.c0, q, M)
    local = sum(parts[:-1])
    ell, b = O.canonicalise(inst.H, inst.f)
    x = W.random_params(2, 1, 95 + seed)[0]
    cross = O.cross_terms(b, q)
    u = np.random.default_rng(seed).uniform(size=4 * cross * 2)
    psi, outcomes, remote = T.trajectory(local, b, q, x, u)
    assert remote == 2 * cross * 2 == O.remote_cx_estimate(cross, 2) and len(outcomes) == 2 * remote
    d = O.cost_diagonal(inst.H, inst.f, inst.c0)
    assert np.linalg.norm(psi - O.qaoa_state(d, x)) <= 1e-12
