"""GPU tests of the gate-level TeleGate trajectory (qq_telegate_state, through the C ABI).

* The trajectory equals the oracle's gate-level trajectory on the same uniforms: identical
  measurement outcomes and data states within 1e-12 (n = 8..12, 2-3 QPUs, dense real and integer
  couplings);
* every trajectory's data state equals the exact complex128 state of the monolithic and of the
  partitioned evaluation (1e-12), whatever the outcomes: the remote CNOTs reproduce the exact
  result;
* the remote CNOT count is 2 x cross x p;
* validation (no allocation, uniforms outside [0, 1)).
"""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import telegate as T
from paper_2606_26297_amd import native as N
from paper_2606_26297_amd import workloads as W
from paper_2606_26297_amd.qaoa import Problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    N.lib()
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"


def uniforms(count, seed):
    rng = np.random.default_rng(seed)
    u = rng.uniform(size=count)
    # every measurement of the protocol has probability 1/2 of giving 1: keep the uniforms away from it
    bad = np.abs(u - 0.5) < 1e-6
    u[bad] = 0.25
    return u


CASES = [("gauss_n8_M2", lambda: W.dense_gaussian_upper(8, 71), 2, 2),
         ("int_n12_M3", lambda: W.workload1()[0], 3, 1),
         ("reg_n10_M2", lambda: W.regular_graph_qubo(10, 72), 2, 3)]


@pytest.mark.parametrize("name,maker,M,p", CASES, ids=[c[0] for c in CASES])
def test_trajectory_matches_oracle_and_exact_state(name, maker, M, p):
    inst = maker()
    n = inst.H.shape[0]
    pb = Problem(inst.H, inst.f, inst.c0)
    caps = O.balanced_capacities(n, M)
    q = W.contiguous_allocation(n, caps)
    cross, remote = pb.set_allocation(q, M, caps)
    x = W.random_params(p, 1, 73 + n)[0]
    u = uniforms(4 * cross * p, 74 + n)
    psi, outcomes, nrem = N.qq_telegate_state(pb.handle, n, x, u)
    assert nrem == 2 * cross * p == remote * p and outcomes.size == 2 * nrem
    ell, b = O.canonicalise(inst.H, inst.f)
    parts = O.partitioned_diagonals(inst.H, inst.f, inst.c0, q, M)
    ref, ref_out, ref_rem = T.trajectory(sum(parts[:-1]), b, q, x, u)
    assert ref_rem == nrem and list(outcomes) == ref_out
    assert np.linalg.norm(psi - ref) <= 1e-12
    assert np.linalg.norm(psi - pb.state(x, c128=True)) <= 1e-12
    assert np.linalg.norm(psi - pb.state(x, c128=True, partitioned=True)) <= 1e-12
    assert 0 < np.mean(outcomes) < 1  # both outcomes occur


def test_telegate_validation():
    inst = W.dense_gaussian_upper(8, 75)
    pb = Problem(inst.H, inst.f, inst.c0)
    x = W.random_params(1, 1, 76)[0]
    with pytest.raises(N.QQError) as ei:
        N.qq_telegate_state(pb.handle, 8, x, uniforms(8, 1))
    assert ei.value.status == N.QQ_E_ALLOCATION
    cross, _ = pb.set_allocation(W.contiguous_allocation(8, [4, 4]), 2)
    u = uniforms(4 * cross, 2)
    u[3] = 1.0
    with pytest.raises(N.QQError) as ei:
        N.qq_telegate_state(pb.handle, 8, x, u)
    assert ei.value.status == N.QQ_E_INVALID
