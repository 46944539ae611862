"""Seeded synthetic QUBO instances and QAOA parameter sets.

This module only *draws inputs*: dense (H, f, c0) triples in the input form of
eq. (2) of the paper (F(z) = c0 + f^T z + z^T H z) and angle vectors in the
interleaved layout x = [gamma_1, beta_1, ..., gamma_p, beta_p] of the training
objective section.  It contains none of the method's arithmetic (no
canonicalisation, no cost diagonal, no statevector work), so both the HIP path
and the CPU oracle can consume the same inputs without sharing code.

The paper's own instances (the 6-, 12-, 15- and 20-variable cases and the unit
commitment data) are not printed in it; the generators below are shape
stand-ins with the sizes and value distributions of the workloads the paper
studies (dense integer QUBOs, a unit-commitment-shaped real QUBO, a sparse
3-regular graph QUBO, uneven batches, and a large dense real QUBO split over
simulated QPUs).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# Seeds for the five standard workloads: instances use 101..105, parameter draws 201..205.
INSTANCE_SEEDS = {1: 101, 2: 102, 3: 103, 4: 104, 5: 105}
PARAM_SEEDS = {1: 201, 2: 202, 3: 203, 4: 204, 5: 205}


@dataclass
class Instance:
    """A QUBO in the paper's dense input form F(z) = c0 + f^T z + z^T H z."""

    H: np.ndarray  # (n, n) float64, row-major, any (not necessarily symmetric)
    f: np.ndarray  # (n,) float64
    c0: float
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.H.shape[0])


def random_params(p: int, batch: int, seed: int, low: float = 0.0, high: float = np.pi) -> np.ndarray:
    """Angle sets x[b] = [gamma_1, beta_1, ..., gamma_p, beta_p], i.i.d. U[low, high]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(low, high, size=(batch, 2 * p)).astype(np.float64)


def optimizer_draws(p_max: int, random_starts: int, perturbed_starts: int, seed: int, scale: float = 0.1):
    """Random inputs of the depth-progression / multi-start search, laid out depth by depth:
    random points (for p = 1 .. p_max, random_starts vectors of 2p angles, U[0, pi]) and warm-start
    offsets (for p = 2 .. p_max, perturbed_starts vectors of 2p values, N(0, scale^2))."""
    rng = np.random.default_rng(seed)
    pts = np.concatenate([rng.uniform(0.0, np.pi, size=random_starts * 2 * p) for p in range(1, p_max + 1)])
    off = [rng.normal(0.0, scale, size=perturbed_starts * 2 * p) for p in range(2, p_max + 1)]
    return pts.astype(np.float64), (np.concatenate(off) if off else np.zeros(0)).astype(np.float64)


def dense_integer_symmetric(n: int, seed: int, lo: int = -10, hi: int = 10) -> Instance:
    """Integer entries drawn from {lo..hi} for i <= j, mirrored to a symmetric H; f = 0, c0 = 0."""
    rng = np.random.default_rng(seed)
    U = rng.integers(lo, hi + 1, size=(n, n)).astype(np.float64)
    U = np.triu(U)
    H = U + np.triu(U, 1).T
    return Instance(H=H, f=np.zeros(n), c0=0.0, name=f"dense_int_sym_n{n}_s{seed}")


def unit_commitment_shaped(n_units: int, seed: int) -> Instance:
    """Unit-commitment-shaped dense real QUBO.

    Objective sum_g c_g x_g + lam * (sum_g P_g x_g - D)^2 with c_g ~ U[10, 50],
    P_g ~ U[20, 100], D = sum(P)/2 and lam = 10 / max(P)^2, written in the
    input form: H = lam * P P^T, f = c - 2 lam D P, c0 = lam D^2.
    """
    rng = np.random.default_rng(seed)
    c = rng.uniform(10.0, 50.0, size=n_units)
    P = rng.uniform(20.0, 100.0, size=n_units)
    D = 0.5 * float(P.sum())
    lam = 10.0 / float(P.max()) ** 2
    H = lam * np.outer(P, P)
    f = c - 2.0 * lam * D * P
    c0 = lam * D * D
    return Instance(H=H, f=f, c0=c0, name=f"uc_shaped_n{n_units}_s{seed}",
                    meta={"c": c, "P": P, "D": D, "lam": lam})


def random_regular_graph(n: int, degree: int, rng: np.random.Generator, max_tries: int = 10000):
    """Uniform-ish random simple d-regular graph by the pairing (configuration) model.

    Stubs are shuffled and paired; a pairing with a self-loop or a repeated
    edge is rejected and redrawn.  Returns a sorted list of (i, j), i < j.
    """
    if (n * degree) % 2:
        raise ValueError("n * degree must be even")
    stubs = np.repeat(np.arange(n), degree)
    for _ in range(max_tries):
        perm = rng.permutation(stubs)
        pairs = perm.reshape(-1, 2)
        ok = True
        seen = set()
        for a, b in pairs:
            if a == b:
                ok = False
                break
            e = (min(a, b), max(a, b))
            if e in seen:
                ok = False
                break
            seen.add(e)
        if ok:
            return sorted((int(a), int(b)) for a, b in seen)
    raise RuntimeError("pairing model did not produce a simple graph")


def regular_graph_qubo(n: int, seed: int, degree: int = 3, lin_sigma: float = 0.5) -> Instance:
    """Sparse QUBO on a random d-regular graph.

    Edge weights w_ij ~ U[0, 1] become the coefficient of z_i z_j (stored in the
    upper triangle H_ij, i < j), linear terms l_i ~ N(0, lin_sigma^2) sit on
    the diagonal H_ii; f = 0, c0 = 0.
    """
    rng = np.random.default_rng(seed)
    edges = random_regular_graph(n, degree, rng)
    w = rng.uniform(0.0, 1.0, size=len(edges))
    lin = rng.normal(0.0, lin_sigma, size=n)
    H = np.zeros((n, n))
    for (i, j), wij in zip(edges, w):
        H[i, j] = wij
    H[np.arange(n), np.arange(n)] = lin
    return Instance(H=H, f=np.zeros(n), c0=0.0, name=f"regular{degree}_n{n}_s{seed}",
                    meta={"edges": edges, "weights": w})


def dense_gaussian_upper(n: int, seed: int) -> Instance:
    """Upper-triangular H with H_ij ~ N(0, 1) for i <= j (not mirrored); f = 0, c0 = 0."""
    rng = np.random.default_rng(seed)
    H = np.triu(rng.normal(0.0, 1.0, size=(n, n)))
    return Instance(H=H, f=np.zeros(n), c0=0.0, name=f"dense_gauss_upper_n{n}_s{seed}")


def separable(n: int, seed: int, scale: float = 1.0) -> Instance:
    """Linear-only instance (no couplings): H diagonal ~ N(0, scale^2), f ~ N(0, scale^2), c0 ~ N(0,1)."""
    rng = np.random.default_rng(seed)
    H = np.diag(rng.normal(0.0, scale, size=n))
    f = rng.normal(0.0, scale, size=n)
    c0 = float(rng.normal())
    return Instance(H=H, f=f, c0=c0, name=f"separable_n{n}_s{seed}")


def cluster_product(block_sizes, seed: int) -> Instance:
    """Block-diagonal couplings: dense N(0,1) upper triangle inside each block, nothing across."""
    rng = np.random.default_rng(seed)
    n = int(sum(block_sizes))
    H = np.zeros((n, n))
    off = 0
    blocks = []
    for m in block_sizes:
        H[off:off + m, off:off + m] = np.triu(rng.normal(0.0, 1.0, size=(m, m)))
        blocks.append((off, m))
        off += m
    c0 = float(rng.normal())
    return Instance(H=H, f=np.zeros(n), c0=c0, name=f"cluster_{'x'.join(map(str, block_sizes))}_s{seed}",
                    meta={"blocks": blocks})


def contiguous_allocation(n: int, capacities) -> np.ndarray:
    """Sequential fill: variables 0.. go to QPU 0 up to its capacity, then QPU 1, and so on."""
    q = np.empty(n, dtype=np.int32)
    i = 0
    for m, cap in enumerate(capacities):
        for _ in range(int(cap)):
            if i < n:
                q[i] = m
                i += 1
    if i != n:
        raise ValueError("capacities do not cover all variables")
    return q


# --- the five standard workloads -------------------------------------------------------------

def workload1():
    """n = 12 dense symmetric integer QUBO, p = 1, one angle pair (0.4, 0.7)."""
    inst = dense_integer_symmetric(12, INSTANCE_SEEDS[1])
    return inst, np.array([[0.4, 0.7]])


def workload2(batch: int = 256, p: int = 4):
    """Unit-commitment-shaped QUBO with 20 units, p = 4, 256 angle sets U[0, pi]."""
    inst = unit_commitment_shaped(20, INSTANCE_SEEDS[2])
    return inst, random_params(p, batch, PARAM_SEEDS[2])


def workload3(batch: int = 64, p: int = 8, n: int = 28):
    """Random 3-regular graph QUBO on 28 nodes, p = 8, 64 multi-start angle sets U[0, pi]."""
    inst = regular_graph_qubo(n, INSTANCE_SEEDS[3])
    return inst, random_params(p, batch, PARAM_SEEDS[3])


def workload4(count: int = 512, n_lo: int = 10, n_hi: int = 22, p_lo: int = 1, p_hi: int = 6):
    """Uneven batch: `count` dense symmetric integer QUBOs, n ~ U{n_lo..n_hi}, p ~ U{p_lo..p_hi}.

    Returns a list of (Instance, params[1, 2p]).
    """
    rng = np.random.default_rng(INSTANCE_SEEDS[4])
    ns = rng.integers(n_lo, n_hi + 1, size=count)
    ps = rng.integers(p_lo, p_hi + 1, size=count)
    seeds = rng.integers(0, 2**31 - 1, size=count)
    prng = np.random.default_rng(PARAM_SEEDS[4])
    out = []
    for k in range(count):
        inst = dense_integer_symmetric(int(ns[k]), int(seeds[k]))
        x = prng.uniform(0.0, np.pi, size=(1, 2 * int(ps[k])))
        out.append((inst, x))
    return out


def workload5(batch: int = 2, p: int = 2, n: int = 32, qpus: int = 4):
    """n = 32 dense N(0,1) upper-triangular QUBO (496 couplings), p = 2, contiguous 4 x 8 allocation."""
    inst = dense_gaussian_upper(n, INSTANCE_SEEDS[5])
    alloc = contiguous_allocation(n, [n // qpus] * qpus)
    return inst, random_params(p, batch, PARAM_SEEDS[5]), alloc
