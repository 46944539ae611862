"""The guarded evaluation calls (qq_evaluate_guarded, qq_evaluate_many_guarded) through the C ABI.

Each returned gradient must be within tol of the FP64 oracle's, relative to ||g||_inf with no floor,
and within the returned bound; sets kept in complex64 equal qq_evaluate's results bit for bit, and for
one problem the sets flagged complex128 equal the per-pass complex128 path's (many problems recompute
theirs in one persistent complex128 launch, held to the oracle here and in the persistent-launch tests).  Covered: a set with a tiny gradient (forced to
complex128) next to ordinary ones, the partitioned mode, QQ_C128 (every set complex128), energy only
(nothing recomputed), a tighter tolerance, and the argument checks.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2606_26297_amd import native as N
from paper_2606_26297_amd import workloads as W
from paper_2606_26297_amd.qaoa import Problem, evaluate_many_guarded

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    N.lib()
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"


def check_against_oracle(inst, x, e, g, err, tol, sigma):
    d = O.cost_diagonal(inst.H, inst.f, inst.c0)
    for b in range(x.shape[0]):
        er, gr = O.gradient(d, x[b])
        dg = float(np.max(np.abs(g[b] - gr)))
        assert abs(e[b] - er) <= 1e-5 * max(abs(er), sigma), (b, e[b], er)
        assert dg <= tol * np.max(np.abs(gr)), (b, dg / np.max(np.abs(gr)))
        assert dg <= err[b], (b, dg, err[b])


def test_guarded_mixes_complex64_and_complex128_sets():
    # the worst problem of the uneven batch (n = 19, p = 1, gradient 1.1e-4 sigma_C) next to random sets
    inst, x0 = W.workload4()[452]
    pb = Problem(inst.H, inst.f, inst.c0)
    try:
        x = np.vstack([x0, W.random_params(1, 3, 601)])
        e, g, up, err = pb.evaluate_guarded(x, tol=1e-5)
        assert up[0] == 1, "the set with a tiny gradient must be recomputed in complex128"
        e64, g64 = pb.evaluate(x, grad=True)
        e128, g128 = pb.evaluate(x[up == 1], grad=True, c128=True)
        assert np.array_equal(e[up == 0], e64[up == 0]) and np.array_equal(g[up == 0], g64[up == 0])
        # one problem: its flagged sets are recomputed by the per-pass complex128 kernels
        assert np.array_equal(e[up == 1], e128) and np.array_equal(g[up == 1], g128)
        check_against_oracle(inst, x, e, g, err, 1e-5, pb.info.sigma_c)
    finally:
        pb.close()


def test_guarded_partitioned_c128_energy_only_and_tolerance():
    inst = W.dense_integer_symmetric(14, 602)
    pb = Problem(inst.H, inst.f, inst.c0)
    try:
        pb.set_allocation(W.contiguous_allocation(14, [7, 7]), 2, [7, 7])
        x = W.random_params(2, 4, 603)
        sig = pb.info.sigma_c
        e, g, up, err = pb.evaluate_guarded(x, tol=1e-5, partitioned=True)
        check_against_oracle(inst, x, e, g, err, 1e-5, sig)
        # a tighter tolerance flags at least as many sets, and the results still hold it
        e2, g2, up2, err2 = pb.evaluate_guarded(x, tol=1e-9)
        assert np.all(up2 >= up) and np.all(up2 == 1)
        check_against_oracle(inst, x, e2, g2, err2, 1e-9, sig)
        # QQ_C128: every set complex128
        B = x.shape[0]
        e3, g3 = np.empty(B), np.empty((B, 4))
        up3, err3 = np.empty(B, dtype=np.int32), np.empty(B)
        N.qq_evaluate_guarded(pb.handle, 2, B, x, N.QQ_ENERGY | N.QQ_GRAD | N.QQ_C128, 0.0, e3, g3, up3, err3)
        assert np.all(up3 == 1)
        e128, g128 = pb.evaluate(x, grad=True, c128=True)
        assert np.array_equal(e3, e128) and np.array_equal(g3, g128)
        # energy only: nothing is recomputed, bounds are 0
        e4 = np.empty(B)
        up4, err4 = np.full(B, 7, dtype=np.int32), np.full(B, 7.0)
        N.qq_evaluate_guarded(pb.handle, 2, B, x, N.QQ_ENERGY, 1e-5, e4, None, up4, err4)
        assert np.all(up4 == 0) and np.all(err4 == 0.0) and np.array_equal(e4, pb.evaluate(x))
    finally:
        pb.close()


def test_many_guarded_matches_single_guarded_and_rejects_bad_input():
    items = [W.workload4()[k] for k in (452, 0, 1, 2)]
    pbs = [Problem(i.H, i.f, i.c0) for i, _ in items]
    try:
        xs = [x for _, x in items]
        e, g, up, err = evaluate_many_guarded(pbs, xs, tol=1e-5)
        for k, ((inst, x), pb) in enumerate(zip(items, pbs)):
            check_against_oracle(inst, x, e[k], g[k], err[k], 1e-5, pb.info.sigma_c)
        assert up[0][0] == 1
        with pytest.raises(N.QQError) as ei:
            evaluate_many_guarded(pbs, xs, tol=-1.0)
        assert ei.value.status == N.QQ_E_INVALID
        with pytest.raises(N.QQError) as ei:
            N.qq_evaluate_many_guarded([pbs[0].handle], [1], [1], [xs[0]], N.QQ_ENERGY | N.QQ_GRAD | N.QQ_C128,
                                       None, 1e-5, [np.empty(1)], [np.empty((1, 2))])
        assert ei.value.status == N.QQ_E_UNSUPPORTED
        with pytest.raises(N.QQError) as ei:
            N.qq_evaluate_guarded(pbs[0].handle, 1, 1, xs[0], N.QQ_ENERGY | N.QQ_GRAD | N.QQ_OUT_ON_DEVICE, 1e-5,
                                  np.empty(1), np.empty((1, 2)))
        assert ei.value.status == N.QQ_E_UNSUPPORTED
    finally:
        for pb in pbs:
            pb.close()
