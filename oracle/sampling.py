"""TEST INFRASTRUCTURE -- the FP64 CPU oracle of shot sampling and the sampled-solution metrics.

Only tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import this
module; the product never does.  It follows the measurement decoding section of the paper on the
exact distribution P(z) = |psi(z)|^2:

* a shot with uniform u in [0, 1) is the first basis index whose cumulative probability (summed in
  index order) exceeds u times the total (the inverse transform); the uniforms are inputs;
* metrics of a set of shots: the best sampled cost and bitstring (among bitstrings of that cost the
  most frequent, ties to the lower index) and its frequency, the fraction of shots at the best cost,
  the sample mean cost (summed over distinct indices in index order), the fraction of shots within
  an absolute margin of the best cost (the paper leaves the margin open), agreement with the exact
  optimum and the shot fractions at it, and the most frequent bitstrings (ties to the lower index);
* the candidate ranking of the depth-progression / multi-start subsection as a sort key.
"""
from __future__ import annotations

import numpy as np


def inverse_cdf(P, u):
    """Shots for uniforms u: first z with sum_{y <= z} P(y) > u * sum(P)."""
    P = np.asarray(P, dtype=np.float64)
    cdf = np.cumsum(P)
    t = np.asarray(u, dtype=np.float64) * cdf[-1]
    idx = np.searchsorted(cdf, t, side="right")
    last = int(np.flatnonzero(P > 0)[-1])
    return np.minimum(idx, last).astype(np.uint64)


def sample_stats(indices, diag, margin, k, cmin, argmin):
    idx = np.asarray(indices, dtype=np.uint64)
    shots = idx.size
    uniq, cnt = np.unique(idx, return_counts=True)  # ascending index
    cost = np.asarray(diag, dtype=np.float64)[uniq.astype(np.int64)]
    best = float(np.min(cost))
    mean = 0.0
    for c, q in zip(cnt, cost):
        mean += float(c) * float(q)
    bi = None
    for i in range(uniq.size):
        if cost[i] == best and (bi is None or cnt[i] > cnt[bi]):
            bi = i
    at_best = int(np.sum(cnt[cost == best]))
    low = int(np.sum(cnt[cost <= best + margin]))
    order = sorted(range(uniq.size), key=lambda i: (-int(cnt[i]), int(uniq[i])))[:k]
    exact_idx = int(cnt[uniq == np.uint64(argmin)].sum())
    return {
        "shots": shots, "distinct": int(uniq.size), "best_index": int(uniq[bi]), "best_cost": best,
        "best_frequency": cnt[bi] / shots, "best_cost_mass": at_best / shots, "mean_cost": mean / shots,
        "low_cost_mass": low / shots, "exact_cost": float(cmin), "exact_index": int(argmin),
        "matches_exact_cost": int(best == cmin), "matches_exact_index": int(int(uniq[bi]) == int(argmin)),
        "exact_cost_mass": int(np.sum(cnt[cost == cmin])) / shots, "exact_index_frequency": exact_idx / shots,
        "elite_index": uniq[order], "elite_count": cnt[order].astype(np.int64), "elite_cost": cost[order],
    }


def rank_key(stats, use_reference=False):
    """Smaller is better: with a reference, (matches exact cost, matches exact bitstring, shots at
    the exact cost, shots at the exact bitstring), larger first; then the best sampled cost
    (smaller), shots at it (larger), the best bitstring's frequency (larger), the mean (smaller)."""
    key = (stats["best_cost"], -stats["best_cost_mass"], -stats["best_frequency"], stats["mean_cost"])
    if use_reference:
        key = (-stats["matches_exact_cost"], -stats["matches_exact_index"], -stats["exact_cost_mass"],
               -stats["exact_index_frequency"]) + key
    return key
