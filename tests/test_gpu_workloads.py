"""GPU parity on the workload shapes at their full sizes where the oracle allows.

* Unit-commitment-shaped QUBO (20 units, dense real FP64 Q), p = 4, all 256
  parameter sets in one complex64 call: every energy against the complex128 path
  and 16 evenly spaced sets against the FP64 oracle (1e-5 relative, with
  max(|E|, sigma_C) as the scale).
* The multi-QPU shape (dense N(0,1) upper-triangular Q, 4 QPUs, contiguous
  allocation, p = 2) at n = 24: the partitioned complex64 evaluation (local and
  cross phases applied as separate factors) against the monolithic one and the
  oracle's gradient (1e-5), and the partitioned complex128 state against the
  oracle's product of per-part phases (1e-10 in the 2-norm).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2606_26297_amd import native as N
from paper_2606_26297_amd import workloads as W
from paper_2606_26297_amd.qaoa import Problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    N.lib()
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"


def e_rel(e, eref, sigma):
    return float(np.max(np.abs(np.asarray(e) - np.asarray(eref)) / np.maximum(np.abs(eref), sigma)))


def g_rel(g, gref):
    g, gref = np.atleast_2d(g), np.atleast_2d(gref)
    return max(float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)) for a, b in zip(g, gref))


def test_unit_commitment_n20_batch256_energies():
    inst, x = W.workload2()
    assert x.shape == (256, 8)
    pb = Problem(inst.H, inst.f, inst.c0)
    assert pb.info.is_integer == 0 and pb.info.diag_bytes == 8
    sig = pb.info.sigma_c
    e64 = pb.evaluate(x)
    e128 = pb.evaluate(x, c128=True)
    assert e_rel(e64, e128, sig) <= 1e-5
    d = O.cost_diagonal(inst.H, inst.f, inst.c0)
    for b in range(0, 256, 16):
        assert e_rel(e64[b], O.energy(d, x[b]), sig) <= 1e-5, b
        assert e_rel(e128[b], O.energy(d, x[b]), sig) <= 1e-10, b


def test_unit_commitment_n20_gradients_sampled():
    inst, x = W.workload2()
    pb = Problem(inst.H, inst.f, inst.c0)
    e, g = pb.evaluate(x[:32], grad=True)
    d = O.cost_diagonal(inst.H, inst.f, inst.c0)
    for b in (0, 13, 31):
        er, gr = O.gradient(d, x[b])
        assert e_rel(e[b], er, pb.info.sigma_c) <= 1e-5 and g_rel(g[b], gr) <= 1e-5, b


def test_multi_qpu_shape_n24_partitioned_vs_monolithic_and_oracle():
    inst, x, alloc = W.workload5(batch=2, p=2, n=24, qpus=4)
    pb = Problem(inst.H, inst.f, inst.c0)
    caps = O.balanced_capacities(24, 4)
    cross, remote = pb.set_allocation(alloc, 4, caps)
    ell, b = O.canonicalise(inst.H, inst.f)
    assert cross == O.cross_terms(b, alloc) and remote == 2 * cross
    sig = pb.info.sigma_c
    e_mono, g_mono = pb.evaluate(x, grad=True)
    e_part, g_part = pb.evaluate(x, grad=True, partitioned=True)
    assert e_rel(e_part, e_mono, sig) <= 1e-5 and g_rel(g_part, g_mono) <= 1e-5
    d = O.cost_diagonal(inst.H, inst.f, inst.c0)
    er, gr = O.gradient(d, x[0])
    assert e_rel(e_part[0], er, sig) <= 1e-5 and g_rel(g_part[0], gr) <= 1e-5
    parts = O.partitioned_diagonals(inst.H, inst.f, inst.c0, alloc, 4)
    ref = O.qaoa_state_multi(parts, x[0])
    assert np.linalg.norm(pb.state(x[0], c128=True, partitioned=True) - ref) <= 1e-10
