"""Pins of the oracle's shot sampling and sampled-solution metrics (CPU only).

* the inverse transform on a distribution with dyadic probabilities, whose cumulative sums are
  exact, at and around every boundary;
* the empirical frequencies of many shots from a small QAOA state agree with P(z) within five
  binomial standard deviations (the sampler draws from the distribution it is given);
* every metric on a hand-built set of shots with hand-computed values;
* the ranking key orders hand-built candidates the way the paper's criteria do.
"""
import numpy as np

from oracle import oracle as O
from oracle import sampling as S
from paper_2606_26297_amd import workloads as W


def test_inverse_transform_at_exact_boundaries():
    P = np.array([0.125, 0.25, 0.125, 0.5])  # cumulative 0.125, 0.375, 0.5, 1
    u = np.array([0.0, 0.124, 0.125, 0.374, 0.375, 0.4999, 0.5, 0.999])
    assert list(S.inverse_cdf(P, u)) == [0, 0, 1, 1, 2, 2, 3, 3]
    # zero-probability entries are never drawn, and the normalisation is by the given total
    P2 = np.array([0.0, 0.5, 0.0, 1.5])
    assert list(S.inverse_cdf(P2, [0.0, 0.2499, 0.25, 0.9])) == [1, 1, 3, 3]


def test_empirical_frequencies_follow_the_distribution():
    inst = W.dense_gaussian_upper(5, 41)
    d = O.cost_diagonal(inst.H, inst.f, inst.c0)
    P = O.probabilities(O.qaoa_state(d, W.random_params(2, 1, 42)[0]))
    shots = 200_000
    u = np.random.default_rng(43).uniform(0.0, 1.0, size=shots)
    counts = np.bincount(S.inverse_cdf(P, u).astype(np.int64), minlength=P.size)
    sd = np.sqrt(shots * P * (1 - P))
    assert np.all(np.abs(counts - shots * P) <= 5 * sd + 1)


def test_metrics_on_hand_built_shots():
    diag = np.array([3.0, -1.0, 2.0, -1.0, 0.0, 5.0, -0.5, 4.0])
    shots = np.array([1, 3, 3, 6, 6, 6, 2, 2, 0, 3], dtype=np.uint64)
    st = S.sample_stats(shots, diag, margin=0.5, k=3, cmin=-1.0, argmin=1)
    assert st["distinct"] == 5 and st["best_cost"] == -1.0
    assert st["best_index"] == 3 and st["best_frequency"] == 0.3  # index 3 (3 shots) beats index 1 (1 shot)
    assert st["best_cost_mass"] == 0.4  # indices 1 and 3
    assert st["low_cost_mass"] == 0.7  # cost <= -0.5: indices 1, 3, 6
    assert abs(st["mean_cost"] - (-1.0 - 3.0 - 1.5 + 4.0 + 3.0) / 10) <= 1e-15
    assert st["matches_exact_cost"] == 1 and st["matches_exact_index"] == 0
    assert st["exact_cost_mass"] == 0.4 and st["exact_index_frequency"] == 0.1
    assert list(st["elite_index"]) == [3, 6, 2] and list(st["elite_count"]) == [3, 3, 2]
    assert list(st["elite_cost"]) == [-1.0, -0.5, 2.0]


def test_rank_key_follows_the_criteria():
    a = {"best_cost": -2.0, "best_cost_mass": 0.1, "best_frequency": 0.1, "mean_cost": 1.0,
         "matches_exact_cost": 0, "matches_exact_index": 0, "exact_cost_mass": 0.0, "exact_index_frequency": 0.0}
    b = dict(a, best_cost=-1.0)                    # worse best cost
    c = dict(a, best_cost_mass=0.2)                # same best cost, more shots at it
    d = dict(a, mean_cost=0.5)                     # tie on the first three, lower mean
    e = dict(b, matches_exact_cost=1)              # with a reference: matching the optimum comes first
    order = sorted(["a", "b", "c", "d"], key=lambda n: S.rank_key({"a": a, "b": b, "c": c, "d": d}[n]))
    assert order == ["c", "d", "a", "b"]
    assert S.rank_key(e, True) < S.rank_key(a, True) and S.rank_key(e) > S.rank_key(a)
