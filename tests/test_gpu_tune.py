"""GPU tests of pinned schedules and the autotuner (through the C ABI).

* workgroups per state and the tile order only change which workgroup takes
  which tile: results agree to 1e-12 relative (order of the FP64 partial sums);
* the set pairing and the set order change which qubits share a pass and where
  the phase is applied between two mixers, hence the complex64 rounding: every
  (pairing, set order) is checked against the closed form of a separable n = 28
  problem (1e-5 relative) and, on a coupled n = 28 instance (which exercises every
  pairing's per-tile cost tables), against the complex128 path, which reads the
  cost diagonal (energy 1e-5 relative, gradient within the stated complex64 bound);
* the autotuner pins a schedule that then evaluates correctly (oracle, 1e-5),
  writes its JSON-lines cache and reads it back without timing.
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2606_26297_amd import native as N
from paper_2606_26297_amd import workloads as W
from paper_2606_26297_amd.qaoa import Problem, evaluate_many

pytestmark = pytest.mark.gpu

GRAD = N.QQ_ENERGY | N.QQ_GRAD


@pytest.fixture(scope="module", autouse=True)
def _lib():
    N.lib()
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def test_workgroups_per_state_and_tile_order_only_reorder_sums():
    inst = W.regular_graph_qubo(20, 51)
    pb = Problem(inst.H, inst.f, inst.c0)
    p, B = 3, 4
    x = W.random_params(p, B, 52)
    e0, g0 = pb.evaluate(x, grad=True)
    for G in (1, 2, 64, 256):
        for order in (0, 1):
            N.qq_set_schedule(pb.handle, p, B, GRAD, {"workgroups_per_state": G, "tile_order": order})
            got = N.qq_get_schedule(pb.handle, p, B, GRAD)
            assert got["workgroups_per_state"] == G and got["tile_order"] == order
            e, g = pb.evaluate(x, grad=True)
            assert rel(e, e0) <= 1e-12 and rel(g, g0) <= 1e-12, (G, order)
    N.qq_set_schedule(pb.handle, p, B, GRAD, None)
    assert N.qq_get_schedule(pb.handle, p, B, GRAD)["pinned"] == 0


def p1_qubit(ell, x):
    v = np.array([1, 1], dtype=complex) / np.sqrt(2)
    for k in range(len(x) // 2):
        g, b = x[2 * k], x[2 * k + 1]
        v = np.array([1, np.exp(-1j * g * ell)]) * v
        v = np.array([[np.cos(b), -1j * np.sin(b)], [-1j * np.sin(b), np.cos(b)]]) @ v
    return abs(v[1]) ** 2


def test_every_set_pairing_and_order_matches_the_separable_closed_form_at_n28():
    n, p, B = 28, 2, 2
    inst = W.separable(n, 53, scale=0.5)
    pb = Problem(inst.H, inst.f, inst.c0)
    ell, _ = O.canonicalise(inst.H, inst.f)
    x = W.random_params(p, B, 54)
    eref = np.array([inst.c0 + sum(li * p1_qubit(li, xb) for li in ell) for xb in x])
    sig = pb.info.sigma_c
    assert N.qq_get_schedule(pb.handle, p, B, N.QQ_ENERGY)["set_order"] == 1  # the default at n = 28
    for pairing in (0, 1, 2):
        for set_order in (0, 1):
            N.qq_set_schedule(pb.handle, p, B, N.QQ_ENERGY,
                              {"workgroups_per_state": 256, "set_pairing": pairing, "set_order": set_order})
            e = pb.evaluate(x)
            assert np.max(np.abs(e - eref) / np.maximum(np.abs(eref), sig)) <= 1e-5, (pairing, set_order)


def test_every_set_pairing_and_order_on_a_coupled_n28_instance_vs_complex128():
    n, p, B = 28, 2, 2
    inst = W.dense_gaussian_upper(n, 56)  # every pair coupled: every table entry sums many terms
    pb = Problem(inst.H, inst.f, inst.c0)
    x = W.random_params(p, B, 57)
    sig = pb.info.sigma_c
    e128, g128 = pb.evaluate(x, grad=True, c128=True)
    for pairing in (0, 1, 2):
        for set_order in (0, 1):
            N.qq_set_schedule(pb.handle, p, B, GRAD,
                              {"workgroups_per_state": 256, "set_pairing": pairing, "set_order": set_order})
            e, g = pb.evaluate(x, grad=True)
            assert np.max(np.abs(e - e128) / np.maximum(np.abs(e128), sig)) <= 1e-5, (pairing, set_order)
            for b in range(B):
                gmax = np.max(np.abs(g128[b]))
                bound = N.QQ_GUARD_REL * gmax + N.QQ_GUARD_K * 2.0 ** -24 * sig ** 2 * 2.0 ** (-n / 2)
                assert np.max(np.abs(g[b] - g128[b])) <= bound, (pairing, set_order, b)


def test_invalid_schedules_are_rejected():
    inst = W.regular_graph_qubo(20, 55)
    pb = Problem(inst.H, inst.f, inst.c0)
    for bad in ({"workgroups_per_state": 3}, {"workgroups_per_state": 512}, {"workgroups_per_state": 0},
                {"workgroups_per_state": 4, "set_pairing": 1}, {"workgroups_per_state": 4, "set_pairing": 3},
                {"workgroups_per_state": 4, "tile_order": 2}, {"workgroups_per_state": 4, "set_order": 2},
                {"workgroups_per_state": 4, "set_order": 1}):  # n = 20 has two sets
        with pytest.raises(N.QQError) as ei:
            N.qq_set_schedule(pb.handle, 2, 2, GRAD, bad)
        assert ei.value.status == N.QQ_E_INVALID, bad


def test_autotune_pins_a_correct_schedule_and_uses_its_cache(tmp_path):
    inst = W.regular_graph_qubo(20, 56)
    pb = Problem(inst.H, inst.f, inst.c0)
    p, B = 3, 4
    cache = str(tmp_path / "tune.jsonl")
    s1 = N.qq_autotune(pb.handle, p, B, GRAD, cache)
    assert s1["from_cache"] == 0 and s1["tried"] >= 2 and s1["ms"] > 0
    got = N.qq_get_schedule(pb.handle, p, B, GRAD)
    assert got["pinned"] == 1 and got["workgroups_per_state"] == s1["workgroups_per_state"]
    lines = [json.loads(line) for line in open(cache)]
    assert len(lines) == 1 and lines[0]["G"] == s1["workgroups_per_state"] and lines[0]["n"] == 20
    # a fresh handle reads the cache without timing
    pb2 = Problem(inst.H, inst.f, inst.c0)
    s2 = N.qq_autotune(pb2.handle, p, B, GRAD, cache)
    assert s2["from_cache"] == 1 and s2["workgroups_per_state"] == s1["workgroups_per_state"]
    assert len(open(cache).readlines()) == 1
    x = W.random_params(p, B, 57)
    e, g = pb2.evaluate(x, grad=True)
    d = O.cost_diagonal(inst.H, inst.f, inst.c0)
    for b in range(B):
        er, gr = O.gradient(d, x[b])
        assert abs(e[b] - er) / max(abs(er), pb.info.sigma_c) <= 1e-5
        assert rel(g[b], gr) <= 1e-5


def test_autotune_many_returns_working_options(tmp_path):
    items = [(W.dense_integer_symmetric(n, 60 + n), W.random_params(1 + n % 3, 1, 70 + n)) for n in range(10, 19)]
    pbs = [Problem(i.H, i.f, i.c0) for i, _ in items]
    xs = [x for _, x in items]
    ps = [x.shape[1] // 2 for x in xs]
    cache = str(tmp_path / "many.jsonl")
    opt, ms = N.qq_autotune_many([pb.handle for pb in pbs], ps, [1] * len(pbs), GRAD, cache)
    assert opt["tiles_per_chunk"] in (4, 8, 16, 32, 64) and ms > 0
    opt2, ms2 = N.qq_autotune_many([pb.handle for pb in pbs], ps, [1] * len(pbs), GRAD, cache)
    assert opt2 == opt and ms2 == pytest.approx(ms, rel=1e-3)
    assert len(open(cache).readlines()) == 1
    e0, g0 = evaluate_many(pbs, xs, grad=True)
    e1, g1 = evaluate_many(pbs, xs, grad=True, options=opt)
    for k in range(len(pbs)):
        assert rel(e1[k], e0[k]) <= 1e-9 and rel(g1[k], g0[k]) <= 1e-9
