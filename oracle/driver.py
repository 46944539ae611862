"""TEST INFRASTRUCTURE -- the FP64 CPU oracle of the depth-progression / multi-start search.

Only tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import this
module; the product never does.  It follows Alg. 1 and the depth-progression / multi-start
subsection of the paper on the exact objective (eq. (15), (17)), with the exact adjoint gradient of
``oracle.gradient`` in place of the paper's SPSA estimate and Adam as the optimisation section
states it:

* for p = 1 .. p_max: the starts of depth p are the lifted best vector of depth p - 1 (if kept),
  perturbed copies of it, then random points (random numbers are inputs, drawn by the caller);
* every start takes ``iterations`` Adam steps of the exact energy;
* every start's final vector is evaluated once more (the paper's final evaluation, here exact) and
  the starts are ranked by that energy, ties to the lower start index; the best is the depth's
  representative;
* the representatives are ranked the same way, ties to the lower depth.

Lifting, which the paper leaves open, is linear interpolation of the gamma and beta sequences onto
one more point (the INTERP rule of Zhou et al., Phys. Rev. X 10, 021067 (2020)).  Ranking by the
exact energy replaces the sampled criteria of the paper's ranking (best sampled cost first), which
need shots.
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as O


def lift(x, p):
    """Interleaved [g1, b1, ..., gp, bp] -> depth p + 1: y_i = (i-1)/p x_{i-1} + (p-i+1)/p x_i,
    i = 1 .. p + 1, x_0 = x_{p+1} = 0, for gamma and beta separately."""
    x = np.asarray(x, dtype=np.float64).reshape(p, 2)
    padded = np.vstack([np.zeros((1, 2)), x, np.zeros((1, 2))])  # rows 0 .. p + 1
    y = np.empty((p + 1, 2))
    for i in range(1, p + 2):
        y[i - 1] = (i - 1) / p * padded[i - 1] + (p - i + 1) / p * padded[i]
    return y.reshape(-1)


def adam_run(diag, x0, iterations, lr, beta1, beta2, eps):
    """Adam on the exact energy from x0: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
    x -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)."""
    x = np.array(x0, dtype=np.float64)
    m = np.zeros_like(x)
    v = np.zeros_like(x)
    for t in range(1, iterations + 1):
        _, g = O.gradient(diag, x)
        m = beta1 * m + (1.0 - beta1) * g
        v = beta2 * v + (1.0 - beta2) * g * g
        x = x - lr * (m / (1.0 - beta1 ** t)) / (np.sqrt(v / (1.0 - beta2 ** t)) + eps)
    return x


def first_lowest(values):
    """Index of the smallest value, ties to the lower index."""
    best = 0
    for i in range(1, len(values)):
        if values[i] < values[best]:
            best = i
    return best


def optimize(diag, p_max, iterations, random_points, perturbations=None, random_starts=1, perturbed_starts=0,
             include_warm=1, adam=(0.01, 0.9, 0.999, 1e-8)):
    """Returns (best_depth, best_start, best_energy, depth_params [p_max][2 p_max], depth_energy,
    start_energy per depth).  random_points / perturbations laid out depth by depth as in the
    library's documentation."""
    lr, b1, b2, eps = adam
    rp = np.asarray(random_points, dtype=np.float64).ravel()
    pt = None if perturbations is None else np.asarray(perturbations, dtype=np.float64).ravel()
    ro = po = 0
    prev = None
    depth_params = np.zeros((p_max, 2 * p_max))
    depth_energy = np.zeros(p_max)
    depth_start = []
    start_energy = []
    for p in range(1, p_max + 1):
        starts = []
        if p >= 2:
            warm = lift(prev, p - 1)
            if include_warm:
                starts.append(warm.copy())
            for _ in range(perturbed_starts):
                starts.append(warm + pt[po:po + 2 * p])
                po += 2 * p
        for _ in range(random_starts):
            starts.append(rp[ro:ro + 2 * p].copy())
            ro += 2 * p
        finals = [adam_run(diag, x0, iterations, lr, b1, b2, eps) for x0 in starts]
        energies = np.array([O.energy(diag, xf) for xf in finals])
        b = first_lowest(energies)
        prev = finals[b]
        depth_params[p - 1, :2 * p] = prev
        depth_energy[p - 1] = energies[b]
        depth_start.append(b)
        start_energy.append(energies)
    d = first_lowest(depth_energy)
    return d + 1, depth_start[d], depth_energy[d], depth_params, depth_energy, start_energy
