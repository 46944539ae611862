"""GPU parity of the depth-progression / multi-start search (qq_optimize, through the C ABI)
against the oracle's search (oracle/driver.py) on the same seeded random inputs.

* complex128: representatives' energies within 1e-9 of the oracle's (relative to max(|E|, sigma_C)),
  their parameters within 1e-7; the chosen start of every depth and the chosen depth equal the
  oracle's wherever the oracle's margin to the runner-up exceeds 1e-7 relative;
* complex64: energies within 1e-5, parameters within 1e-4 (Adam carries the complex64 gradient
  error of about 1e-6 through the iterations), choices compared where the margin exceeds 1e-3;
* the partitioned complex128 search equals the monolithic one (1e-9);
* option and input validation.
"""
import numpy as np
import pytest

from oracle import driver as D
from oracle import oracle as O
from paper_2606_26297_amd import native as N
from paper_2606_26297_amd import workloads as W
from paper_2606_26297_amd.qaoa import Problem

pytestmark = pytest.mark.gpu

ADAM = (0.05, 0.9, 0.999, 1e-8)


@pytest.fixture(scope="module", autouse=True)
def _lib():
    N.lib()
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"


def margin_ok(values, idx, rel):
    """True when the chosen index beats every other value by more than rel * scale."""
    v = np.asarray(values, dtype=float)
    if len(v) == 1:
        return True
    others = np.delete(v, idx)
    return np.min(others) - v[idx] > rel * max(1.0, np.max(np.abs(v)))


CASES = [("n10_gauss", lambda: W.dense_gaussian_upper(10, 21)), ("n14_reg", lambda: W.regular_graph_qubo(14, 22))]


@pytest.mark.parametrize("name,maker", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("c128", [True, False], ids=["c128", "c64"])
def test_search_matches_oracle(name, maker, c128):
    inst = maker()
    pb = Problem(inst.H, inst.f, inst.c0)
    d = O.cost_diagonal(inst.H, inst.f, inst.c0)
    p_max, iters, R, P = 3, 12, 3, 2
    pts, off = W.optimizer_draws(p_max, R, P, 100 + inst.n)
    opts = {"p_max": p_max, "iterations": iters, "random_starts": R, "perturbed_starts": P, "include_warm": 1,
            "flags": N.QQ_C128 if c128 else 0, "adam": ADAM}
    got = N.qq_optimize(pb.handle, opts, pts, off)
    bd, bs, be, dp, de, se = D.optimize(d, p_max, iters, pts, off, random_starts=R, perturbed_starts=P,
                                        include_warm=1, adam=ADAM)
    sig = pb.info.sigma_c
    etol, xtol, mrel = (1e-9, 1e-7, 1e-7) if c128 else (1e-5, 1e-4, 1e-3)
    assert got["steps"] == sum(len(e) for e in se) * iters
    for p in range(p_max):
        assert len(got["start_energy"][p]) == len(se[p])
        assert np.max(np.abs(got["start_energy"][p] - se[p])) <= etol * max(np.max(np.abs(se[p])), sig), p
        ref_b = int(np.argmin(se[p]))
        if margin_ok(se[p], ref_b, mrel):
            assert int(np.argmin(got["start_energy"][p])) == ref_b, p
            assert np.max(np.abs(got["depth_params"][p] - dp[p])) <= xtol, p
        assert abs(got["depth_energy"][p] - de[p]) <= etol * max(abs(de[p]), sig), p
    if margin_ok(de, bd - 1, mrel):
        assert got["best_depth"] == bd
        if margin_ok(se[bd - 1], bs, mrel):
            assert got["best_start"] == bs
    assert abs(got["best_energy"] - be) <= etol * max(abs(be), sig)
    assert got["best_energy"] >= d.min() - 1e-9 * sig


def test_partitioned_search_equals_monolithic():
    inst = W.dense_gaussian_upper(12, 23)
    pb = Problem(inst.H, inst.f, inst.c0)
    caps = O.balanced_capacities(12, 3)
    pb.set_allocation(W.contiguous_allocation(12, caps), 3, caps)
    pts, off = W.optimizer_draws(2, 2, 1, 24)
    opts = {"p_max": 2, "iterations": 8, "random_starts": 2, "perturbed_starts": 1, "adam": ADAM,
            "flags": N.QQ_C128}
    a = N.qq_optimize(pb.handle, opts, pts, off)
    b = N.qq_optimize(pb.handle, dict(opts, flags=N.QQ_C128 | N.QQ_PARTITIONED), pts, off)
    assert np.max(np.abs(a["depth_energy"] - b["depth_energy"])) <= 1e-9 * pb.info.sigma_c
    assert np.max(np.abs(a["depth_params"] - b["depth_params"])) <= 1e-8
    assert (a["best_depth"], a["best_start"]) == (b["best_depth"], b["best_start"])


def test_search_validation():
    inst = W.regular_graph_qubo(10, 25)
    pb = Problem(inst.H, inst.f, inst.c0)
    pts, off = W.optimizer_draws(2, 1, 1, 26)
    base = {"p_max": 2, "iterations": 2, "random_starts": 1, "perturbed_starts": 1}
    pts65, off65 = W.optimizer_draws(N.QQ_MAX_P + 1, 1, 1, 27)
    cases = [({"p_max": 0, "perturbed_starts": 0}, np.zeros(0), None),
             ({"p_max": N.QQ_MAX_P + 1}, pts65, off65),
             ({"random_starts": 0}, np.zeros(0), off),
             ({"iterations": -1}, pts, off), ({"include_warm": 2}, pts, off), ({"flags": N.QQ_GRAD}, pts, off),
             ({"adam": (0.0, 0.9, 0.999, 1e-8)}, pts, off)]
    for bad, rp, pt in cases:
        with pytest.raises(N.QQError) as ei:
            N.qq_optimize(pb.handle, dict(base, **bad), rp, pt)
        assert ei.value.status == N.QQ_E_INVALID, bad
    nan_pts, inf_off = pts.copy(), off.copy()
    nan_pts[3] = np.nan
    inf_off[1] = np.inf
    for rp, pt in ((nan_pts, off), (pts, inf_off)):
        with pytest.raises(N.QQError) as ei:
            N.qq_optimize(pb.handle, base, rp, pt)
        assert ei.value.status == N.QQ_E_INVALID
    with pytest.raises(ValueError):
        N.qq_optimize(pb.handle, base, pts[:-1], off)
