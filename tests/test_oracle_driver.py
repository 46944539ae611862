"""Pins of the oracle's depth-progression / multi-start search (CPU only).

Each check ties the oracle to a fact that does not come from its own code path:
* the lifting rule maps samples of a linear function of the layer index onto samples of the same
  function on the finer grid (the defining property of linear interpolation), and duplicates a
  single layer;
* the first Adam step from zero moments has the closed form x - lr g / (|g| + eps) (bias-corrected
  m = g and v = g^2), with g from central finite differences of the energy;
* every final energy respects the variational bound E >= min_z C(z) (brute force), and on one qubit,
  where E(gamma, beta) = c0 + (l/2)(1 + sin 2beta sin gamma l), the search reaches min C;
* with a zero cost every energy is exactly 0 and the zero gradient leaves the points unchanged, so
  the ranking's tie rule alone picks depth 1, start 0;
* the first start of depth 2 is the lifted depth-1 representative: with zero iterations its final
  energy is the energy of that lifted vector.
"""
import numpy as np
import pytest

from oracle import driver as D
from oracle import oracle as O
from paper_2606_26297_amd import workloads as W


@pytest.mark.parametrize("p", [2, 3, 5, 8])
def test_lift_maps_linear_sequences_to_linear_sequences(p):
    a = np.array([0.3, -0.2])
    b = np.array([1.1, 0.7])
    x = np.stack([a + b * (i - 1) / (p - 1) for i in range(1, p + 1)]).reshape(-1)
    y = D.lift(x, p).reshape(p + 1, 2)
    want = np.stack([a + b * (i - 1) / p for i in range(1, p + 2)])
    assert np.max(np.abs(y - want)) <= 1e-14


def test_lift_duplicates_a_single_layer():
    assert np.array_equal(D.lift([0.4, 1.3], 1), np.array([0.4, 1.3, 0.4, 1.3]))


def test_first_adam_step_closed_form():
    inst = W.regular_graph_qubo(8, 3)
    d = O.cost_diagonal(inst.H, inst.f, inst.c0)
    x0 = W.random_params(2, 1, 4)[0]
    lr, eps = 0.05, 1e-8
    g = O.fd_gradient(d, x0)
    x1 = D.adam_run(d, x0, 1, lr, 0.9, 0.999, eps)
    assert np.max(np.abs(x1 - (x0 - lr * g / (np.abs(g) + eps)))) <= 1e-8


def test_variational_bound_and_one_qubit_optimum():
    ell, c0 = 1.7, -0.4
    d = O.cost_diagonal(np.array([[ell]]), None, c0)
    assert d.min() == c0  # z = 0 costs c0 < c0 + ell
    pts, _ = W.optimizer_draws(1, 3, 0, 5)
    best_depth, best_start, best_e, _, _, se = D.optimize(d, 1, 400, pts, random_starts=3, adam=(0.05, 0.9, 0.999, 1e-8))
    assert best_depth == 1 and np.all(se[0] >= c0 - 1e-12)
    assert abs(best_e - c0) <= 1e-6
    # and on a coupled instance: every final energy is above the brute-force minimum
    inst = W.dense_gaussian_upper(7, 6)
    d = O.cost_diagonal(inst.H, inst.f, inst.c0)
    pts, off = W.optimizer_draws(2, 2, 1, 7)
    *_, se = D.optimize(d, 2, 10, pts, off, random_starts=2, perturbed_starts=1)
    assert all(np.all(e >= d.min() - 1e-12) for e in se)


def test_zero_cost_ties_go_to_depth_one_start_zero():
    d = O.cost_diagonal(np.zeros((3, 3)), None, 0.0)
    pts, off = W.optimizer_draws(3, 2, 2, 8)
    best_depth, best_start, best_e, dparams, de, se = D.optimize(d, 3, 5, pts, off, random_starts=2,
                                                                perturbed_starts=2)
    assert (best_depth, best_start) == (1, 0) and best_e == 0.0
    assert np.all(de == 0.0) and all(np.all(e == 0.0) for e in se)
    assert np.array_equal(dparams[0, :2], pts[:2])  # zero gradient: the first random point is unchanged


def test_warm_start_is_the_lifted_representative():
    inst = W.regular_graph_qubo(6, 9)
    d = O.cost_diagonal(inst.H, inst.f, inst.c0)
    pts, _ = W.optimizer_draws(2, 1, 0, 10)
    _, _, _, dparams, de, se = D.optimize(d, 2, 0, pts, random_starts=1, include_warm=1)
    warm = D.lift(dparams[0, :2], 1)
    assert se[1][0] == pytest.approx(O.energy(d, warm), abs=1e-13)
