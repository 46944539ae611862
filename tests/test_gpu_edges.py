"""Edge cases of the follow-up entry points (through the C ABI), against the oracle.

* shots at tiny sizes (n = 1, 3, 6: fewer amplitudes than one row of a block), at n = 12 (one
  block) and n = 13 (two blocks), complex128: every shot equals the oracle's inverse transform;
* the search with zero Adam steps: every start keeps its point, so the representatives are the
  lowest-energy given points (depth 1) and the lifted points (depth 2), as in the oracle;
* a TeleGate trajectory with one QPU (no cross couplings, no remote CNOTs, no uniforms) equals the
  exact state; the allocation helpers with one variable per QPU.
"""
import numpy as np
import pytest

from oracle import allocation as A
from oracle import driver as D
from oracle import oracle as O
from oracle import sampling as S
from paper_2606_26297_amd import native as N
from paper_2606_26297_amd import workloads as W
from paper_2606_26297_amd.qaoa import Problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    N.lib()
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"


@pytest.mark.parametrize("n", [1, 3, 6, 12, 13])
def test_shots_at_small_sizes(n):
    inst = W.dense_gaussian_upper(n, 700 + n)
    pb = Problem(inst.H, inst.f, inst.c0)
    d = O.cost_diagonal(inst.H, inst.f, inst.c0)
    x = W.random_params(2, 1, 710 + n)[0]
    P = O.probabilities(O.qaoa_state(d, x))
    u = np.random.default_rng(720 + n).uniform(size=2000)
    z = pb.sample(x, u, c128=True)
    ref = S.inverse_cdf(P, u)
    cdf = np.cumsum(P)
    t = u * cdf[-1]
    # equal to the oracle except where the target lies within rounding of a boundary
    near = np.min(np.abs(t[:, None] - cdf[None, :]), axis=1) <= 1e-12
    assert np.all((z == ref) | near)


def test_search_with_zero_steps_ranks_the_given_points():
    inst = W.regular_graph_qubo(12, 730)
    pb = Problem(inst.H, inst.f, inst.c0)
    d = O.cost_diagonal(inst.H, inst.f, inst.c0)
    pts, off = W.optimizer_draws(2, 3, 2, 731)
    opts = {"p_max": 2, "iterations": 0, "random_starts": 3, "perturbed_starts": 2, "flags": N.QQ_C128}
    got = N.qq_optimize(pb.handle, opts, pts, off)
    bd, bs, be, dp, de, se = D.optimize(d, 2, 0, pts, off, random_starts=3, perturbed_starts=2)
    assert got["steps"] == 0
    assert np.array_equal(got["depth_params"][0, :2], pts[2 * int(np.argmin(se[0])):][:2])
    assert np.max(np.abs(got["depth_params"] - dp)) <= 1e-15
    for p in range(2):
        assert np.max(np.abs(got["start_energy"][p] - se[p])) <= 1e-11 * max(1.0, np.max(np.abs(se[p])))
    assert (got["best_depth"], got["best_start"]) == (bd, bs)


def test_telegate_with_one_qpu_and_allocation_extremes():
    inst = W.dense_gaussian_upper(8, 740)
    pb = Problem(inst.H, inst.f, inst.c0)
    cross, remote = pb.set_allocation(np.zeros(8, dtype=np.int32), 1)
    assert cross == 0 and remote == 0
    x = W.random_params(2, 1, 741)[0]
    psi, outcomes, nrem = N.qq_telegate_state(pb.handle, 8, x, np.zeros(0))
    assert nrem == 0 and outcomes.size == 0
    assert np.linalg.norm(psi - pb.state(x, c128=True)) <= 1e-12
    # one variable per QPU: every coupling crosses
    q, xg = N.qq_allocation(inst.H, 8, strategy=N.QQ_ALLOC_GRAPH)
    assert sorted(q) == list(range(8)) and xg == A.cross_count(inst.H, list(q)) == 28
