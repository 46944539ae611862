"""GPU parity of the persistent many-problem launch (qq_evaluate_many) through the C ABI.

References: the FP64 oracle (energy and adjoint gradient) on every problem of the mixed
set, and its stored values for all 512 problems of the uneven batch; per-problem
qq_evaluate calls (the per-launch path).
Tolerances: 1e-5 relative against the oracle (energy |dE| / max(|E|, sigma_C),
gradient ||dg||_inf / ||g||_inf); 1e-9 relative against qq_evaluate for n >= 13
(same complex64 arithmetic per amplitude, only the order of the FP64 partial sums
differs) and 1e-5 for n <= 12 (a different single-tile kernel); bit-identical
results across grid sizes (fixed-order reductions).  Complex128 states (QQ_C128):
1e-10 against the oracle, 1e-11 against per-problem complex128 calls.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2606_26297_amd import native as N
from paper_2606_26297_amd import workloads as W
from paper_2606_26297_amd.qaoa import Problem, evaluate_many, evaluate_many_guarded

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    N.lib()
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"


def e_err(e, eref, sigma):
    return float(np.max(np.abs(np.asarray(e) - np.asarray(eref)) / np.maximum(np.abs(eref), sigma)))


def g_err(g, gref):
    g, gref = np.atleast_2d(g), np.atleast_2d(gref)
    return max(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300) for a, b in zip(g, gref))


# uneven mix: single-tile sizes (n <= 12, incl. n < 4), two-set and three-set plans,
# full and partial high sets, integer (int16 / int32) and real diagonals
MIX = [(1, 2, 1), (3, 1, 2), (7, 3, 1), (11, 2, 2), (12, 4, 1), (13, 1, 1), (14, 3, 2), (16, 2, 1),
       (17, 5, 1), (19, 2, 1), (20, 3, 2), (21, 2, 1), (22, 1, 1)]


def mix_instances():
    out = []
    for k, (n, p, B) in enumerate(MIX):
        if k % 3 == 0:
            inst = W.dense_gaussian_upper(n, 300 + k)        # real FP64 diagonal
        elif k % 3 == 1:
            inst = W.dense_integer_symmetric(n, 300 + k)     # int16 diagonal
        else:
            inst = W.Instance(H=np.triu(np.random.default_rng(300 + k).integers(-3000, 3001, (n, n))).astype(float),
                              f=np.zeros(n), c0=5.0)          # int32 diagonal
        out.append((inst, W.random_params(p, B, 400 + k)))
    return out


@pytest.fixture(scope="module")
def mix():
    insts = mix_instances()
    pbs = [Problem(i.H, i.f, i.c0) for i, _ in insts]
    return insts, pbs


def test_mix_covers_every_diagonal_type(mix):
    _, pbs = mix
    assert sorted({pb.info.diag_bytes for pb in pbs}) == [2, 4, 8]


def per_problem_same_order(pb, x):
    """pb.evaluate with the set order of the persistent launch (the qubit-0..11 set first), so the two
    paths run the same complex64 operations."""
    p, B = x.shape[1] // 2, x.shape[0]
    flags = N.QQ_ENERGY | N.QQ_GRAD
    G = N.qq_get_schedule(pb.handle, p, B, flags)["workgroups_per_state"]
    N.qq_set_schedule(pb.handle, p, B, flags, {"workgroups_per_state": G, "set_order": 0})
    try:
        return pb.evaluate(x, grad=True)
    finally:
        N.qq_set_schedule(pb.handle, p, B, flags, None)


def test_many_vs_oracle_and_per_problem(mix):
    insts, pbs = mix
    xs = [x for _, x in insts]
    e, g = evaluate_many(pbs, xs, grad=True)
    for k, ((inst, x), pb) in enumerate(zip(insts, pbs)):
        n = pb.n
        sig = pb.info.sigma_c
        print(f"problem {k}: n={n} p={x.shape[1] // 2} B={x.shape[0]}", flush=True)
        # per-problem launches (same set order)
        e1, g1 = per_problem_same_order(pb, x)
        tol = 1e-9 if n > 12 else 1e-5
        assert e_err(e[k], e1, sig) <= tol, (k, e[k], e1)
        assert g_err(g[k], g1) <= tol, k
        # oracle (all of these sizes finish in seconds)
        d = O.cost_diagonal(inst.H, inst.f, inst.c0)
        for b in range(x.shape[0]):
            er, gr = O.gradient(d, x[b])
            assert e_err(e[k][b], er, sig) <= 1e-5, (k, b)
            assert g_err(g[k][b], gr) <= 1e-5, (k, b)


def test_many_c128_vs_per_problem_and_oracle(mix):
    """The complex128 launch runs the general pass bodies of the per-pass complex128 kernels: same
    arithmetic per amplitude, only the set order and the order of the FP64 partial sums differ, so
    1e-11 against per-problem complex128 calls; 1e-10 against the oracle (n <= 17)."""
    insts, pbs = mix
    xs = [x for _, x in insts]
    e, g = evaluate_many(pbs, xs, grad=True, c128=True)
    e0, g0 = evaluate_many(pbs, xs, grad=False, c128=True)
    assert g0 is None
    for k, ((inst, x), pb) in enumerate(zip(insts, pbs)):
        sig = pb.info.sigma_c
        print(f"problem {k}: n={pb.n} p={x.shape[1] // 2} B={x.shape[0]}", flush=True)
        e1, g1 = pb.evaluate(x, grad=True, c128=True)
        assert e_err(e[k], e1, sig) <= 1e-11, (k, e[k], e1)
        assert g_err(g[k], g1) <= 1e-11, k
        assert e_err(e0[k], e1, sig) <= 1e-11, k
        if pb.n <= 17:
            d = O.cost_diagonal(inst.H, inst.f, inst.c0)
            for b in range(x.shape[0]):
                er, gr = O.gradient(d, x[b])
                assert e_err(e[k][b], er, sig) <= 1e-10, (k, b)
                assert g_err(g[k][b], gr) <= 1e-10, (k, b)


def test_many_c128_bitwise_across_grids_and_close_across_chunks(mix):
    insts, pbs = mix
    xs = [x for _, x in insts]
    ea, ga = evaluate_many(pbs, xs, grad=True, c128=True)
    eb, gb = evaluate_many(pbs, xs, grad=True, c128=True, options={"max_workgroups": 5})
    ec, gc = evaluate_many(pbs, xs, grad=True, c128=True, options={"tiles_per_chunk": 1})
    ed, gd = evaluate_many(pbs, xs, grad=True, c128=True, options={"max_workgroups": 1})
    for k, pb in enumerate(pbs):
        assert np.array_equal(ea[k], eb[k]) and np.array_equal(ga[k], gb[k]), k
        assert np.array_equal(ea[k], ed[k]) and np.array_equal(ga[k], gd[k]), k
        assert e_err(ec[k], ea[k], pb.info.sigma_c) <= 1e-12, k
        assert g_err(gc[k], ga[k]) <= 1e-12, k


def test_many_energy_only_matches_grad_run(mix):
    insts, pbs = mix
    xs = [x for _, x in insts]
    e_only, g_none = evaluate_many(pbs, xs, grad=False)
    assert g_none is None
    e, _ = evaluate_many(pbs, xs, grad=True)
    for k, pb in enumerate(pbs):
        assert e_err(e_only[k], e[k], pb.info.sigma_c) <= 1e-9, k


def test_many_bitwise_across_grid_sizes_and_repeat(mix):
    insts, pbs = mix
    xs = [x for _, x in insts]
    ea, ga = evaluate_many(pbs, xs, grad=True)
    eb, gb = evaluate_many(pbs, xs, grad=True, options={"max_workgroups": 7})
    ec, gc = evaluate_many(pbs, xs, grad=True)
    # one workgroup takes every item in ticket order: it completes only if every item's
    # dependencies come earlier in that order (otherwise the bounded wait reports QQ_E_DEVICE)
    ed, gd = evaluate_many(pbs, xs, grad=True, options={"max_workgroups": 1})
    for k in range(len(pbs)):
        assert np.array_equal(ea[k], eb[k]) and np.array_equal(ga[k], gb[k]), k
        assert np.array_equal(ea[k], ec[k]) and np.array_equal(ga[k], gc[k]), k
        assert np.array_equal(ea[k], ed[k]) and np.array_equal(ga[k], gd[k]), k


def test_many_chunk_sizes_agree(mix):
    insts, pbs = mix
    xs = [x for _, x in insts]
    ea, ga = evaluate_many(pbs, xs, grad=True, options={"tiles_per_chunk": 1})
    eb, gb = evaluate_many(pbs, xs, grad=True, options={"tiles_per_chunk": 64})
    for k, pb in enumerate(pbs):
        assert e_err(ea[k], eb[k], pb.info.sigma_c) <= 1e-9, k
        assert g_err(ga[k], gb[k]) <= 1e-9, k


def test_many_device_path_matches_host(mix):
    import torch

    insts, pbs = mix
    xs = [x for _, x in insts]
    eh, gh = evaluate_many(pbs, xs, grad=True)
    xt = [torch.tensor(x, device="cuda:0") for x in xs]
    ed, gd = evaluate_many(pbs, xt, grad=True)
    torch.cuda.synchronize()
    for k in range(len(pbs)):
        assert np.array_equal(ed[k].cpu().numpy(), eh[k]) and np.array_equal(gd[k].cpu().numpy(), gh[k]), k


def test_many_rejects_unsupported_and_bad_arguments(mix):
    _, pbs = mix
    x = [W.random_params(1, 1, 1)]
    e = [np.empty(1)]
    g = [np.empty((1, 2))]
    with pytest.raises(N.QQError) as ei:
        N.qq_evaluate_many([pbs[0].handle], [1], [1], x, N.QQ_ENERGY | N.QQ_PARTITIONED, None, None, 0, None, e, g)
    assert ei.value.status == N.QQ_E_UNSUPPORTED
    with pytest.raises(N.QQError) as ei:
        N.qq_evaluate_many([pbs[0].handle], [1], [0], x, N.QQ_ENERGY, None, None, 0, None, e, g)
    assert ei.value.status == N.QQ_E_INVALID
    with pytest.raises(N.QQError) as ei:
        N.qq_evaluate_many([pbs[0].handle], [1], [1], [np.array([[0.1, np.nan]])], N.QQ_ENERGY, None, None, 0, None,
                           e, g)
    assert ei.value.status == N.QQ_E_INVALID
    with pytest.raises(N.QQError) as ei:
        N.qq_evaluate_many([pbs[0].handle], [1], [1], x, N.QQ_ENERGY | N.QQ_GRAD, None, None, 0, None, e, None)
    assert ei.value.status == N.QQ_E_INVALID
    with pytest.raises(N.QQError) as ei:
        N.qq_evaluate_many([pbs[0].handle], [1], [1], x, N.QQ_ENERGY, {"tiles_per_chunk": -1}, None, 0, None, e, g)
    assert ei.value.status == N.QQ_E_INVALID


def test_many_wait_limit_reports_error_then_recovers(mix):
    """A wait limit far below any pass time makes dependency waits run out: the flag
    drains the launch and the call reports QQ_E_DEVICE; a normal call afterwards works."""
    insts, pbs = mix
    big = [k for k, (n, _, _) in enumerate(MIX) if n >= 20]
    sub = [pbs[k] for k in big]
    xs = [insts[k][1] for k in big]
    with pytest.raises(N.QQError) as ei:
        evaluate_many(sub, xs, grad=True, options={"wait_limit_ms": 1e-6})
    assert ei.value.status == N.QQ_E_DEVICE
    e, g = evaluate_many(sub, xs, grad=True)
    for k, pb in zip(big, sub):
        e1, g1 = per_problem_same_order(pb, insts[k][1])
        assert e_err(e[big.index(k)], e1, pb.info.sigma_c) <= 1e-9


def c64_bound(n, sigma, gmax):
    """The library's complex64 gradient error model (QQ_GUARD_REL, QQ_GUARD_K in the header)."""
    return N.QQ_GUARD_REL * gmax + N.QQ_GUARD_K * sigma * sigma * 2.0 ** -24 * 2.0 ** (-0.5 * n)


def test_workload4_many_vs_per_problem_launches():
    """The uneven-batch workload (512 dense integer problems, n in 10..22, p in 1..6): one persistent
    launch against 512 per-problem qq_evaluate calls with the same set order (the same complex64
    operations for n > 12: 1e-9; for n <= 12 the persistent launch evaluates the whole problem in one
    tile and the per-problem call runs the generic single-pass kernel, two complex64 codes: 2e-5)."""
    items = W.workload4()
    pbs = [Problem(i.H, i.f, i.c0) for i, _ in items]
    xs = [x for _, x in items]
    e, g = evaluate_many(pbs, xs, grad=True)
    de, dg = [], []
    for k, ((inst, x), pb) in enumerate(zip(items, pbs)):
        e1, g1 = per_problem_same_order(pb, x)
        de.append(e_err(e[k], e1, pb.info.sigma_c))
        dg.append(g_err(g[k], g1))
    print(f"workload4: many vs per-problem: worst energy rel {max(de):.3e}, worst grad rel {max(dg):.3e}", flush=True)
    for k, pb in enumerate(pbs):
        tol = 1e-9 if pb.n > 12 else 2e-5
        assert de[k] <= tol and dg[k] <= tol, (k, pb.n, de[k], dg[k])


def test_workload4_every_problem_vs_stored_oracle():
    """All 512 problems of the uneven batch against the FP64 oracle's energy and adjoint gradient
    (stored by tests/golden/make_uneven512_oracle.py; energy |dE| / max(|E|, sigma_C), gradient
    ||dg||_inf / ||g||_inf, no floor):
      * the complex64 persistent launch: every energy within 1e-5, and every gradient error within the
        library's stated complex64 bound QQ_GUARD_REL ||g||_inf + QQ_GUARD_K 2^-24 sigma_C^2 2^(-n/2);
      * the guarded evaluation (qq_evaluate_many_guarded): every gradient within 1e-5 relative, the
        sets it keeps in complex64 bit-identical to the persistent launch, and every returned error
        bound at or above the actual error."""
    import json
    import os

    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "uneven512_oracle.json")))["problems"]
    items = W.workload4()
    assert len(ref) == len(items) == 512
    pbs = [Problem(i.H, i.f, i.c0) for i, _ in items]
    xs = [x for _, x in items]
    e, g = evaluate_many(pbs, xs, grad=True)
    eg, gg, up, err = evaluate_many_guarded(pbs, xs, tol=1e-5)
    raw_rel, worst = [], 0.0
    for k, pb in enumerate(pbs):
        r = ref[k]
        assert r["n"] == pb.n and r["p"] == xs[k].shape[1] // 2, k
        sig = pb.info.sigma_c
        gr = np.array(r["gradient"])
        gmax = float(np.max(np.abs(gr)))
        assert e_err(e[k][0], r["energy"], sig) <= 1e-5, (k, e[k][0], r["energy"])
        d_raw = float(np.max(np.abs(g[k][0] - gr)))
        raw_rel.append(d_raw / gmax)
        assert d_raw <= c64_bound(pb.n, sig, gmax), (k, pb.n, d_raw, c64_bound(pb.n, sig, gmax))
        assert e_err(eg[k][0], r["energy"], sig) <= 1e-5, k
        d_g = float(np.max(np.abs(gg[k][0] - gr)))
        worst = max(worst, d_g / gmax)
        assert d_g <= 1e-5 * gmax, (k, pb.n, r["p"], d_g / gmax, int(up[k][0]))
        assert d_g <= err[k][0], (k, d_g, err[k][0])
        if not up[k][0]:
            assert np.array_equal(gg[k], g[k]) and np.array_equal(eg[k], e[k]), k
    n_up = int(sum(int(u[0]) for u in up))
    print(f"workload4 vs oracle: complex64 grad rel max {max(raw_rel):.3e} (median {np.median(raw_rel):.3e}, "
          f"{sum(v > 1e-5 for v in raw_rel)} above 1e-5); guarded: {n_up} sets in complex128, "
          f"grad rel max {worst:.3e}", flush=True)
