"""Workspace poisoning (QQ_POISON=1): every evaluation workspace is filled with all-ones words (NaN in
float and double) before the evaluation's kernels run.  A kernel that read a workspace byte the call
had not written first would turn its results into NaN or change them; the results must instead equal
the unpoisoned ones bit for bit, for the complex64 specialised passes (energy and gradient), the
generic complex128 and single-pass kernels, the persistent many-problem launch and the final state
(n = 24 covers the interleaved psi / lambda region of gradient evaluations).  Also checks QQ_LOG's one
line per call."""
import os

import numpy as np
import pytest

from paper_2606_26297_amd import native as N
from paper_2606_26297_amd import workloads as W
from paper_2606_26297_amd.qaoa import Problem, evaluate_many

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    N.lib()
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"


def run_all(pbs, xs):
    out = []
    for pb, x in zip(pbs, xs):
        out.append(pb.evaluate(x, grad=True))
        out.append(pb.evaluate(x, grad=True, c128=True))
        out.append((pb.state(x[0]),))
    out.append(tuple(evaluate_many(pbs, xs, grad=True)))
    return out


def test_poisoned_workspaces_change_nothing(monkeypatch):
    # n = 24: gradients with psi and lambda interleaved in one region
    insts = [W.dense_integer_symmetric(10, 501), W.regular_graph_qubo(18, 502), W.dense_gaussian_upper(21, 503),
             W.regular_graph_qubo(24, 511)]
    xs = [W.random_params(p, 3, 510 + p) for p in (2, 3, 2, 2)]
    pbs = [Problem(i.H, i.f, i.c0) for i in insts]
    try:
        monkeypatch.delenv("QQ_POISON", raising=False)
        clean = run_all(pbs, xs)
        monkeypatch.setenv("QQ_POISON", "1")
        poisoned = run_all(pbs, xs)
        for a, b in zip(clean, poisoned):
            for u, v in zip(a, b):
                if isinstance(u, list):
                    for uu, vv in zip(u, v):
                        assert np.all(np.isfinite(vv)) and np.array_equal(uu, vv)
                else:
                    assert np.all(np.isfinite(v)) and np.array_equal(u, v)
    finally:
        for pb in pbs:
            pb.close()


def test_call_log_line(capfd, monkeypatch):
    inst = W.dense_integer_symmetric(8, 504)
    pb = Problem(inst.H, inst.f, inst.c0)
    try:
        monkeypatch.setenv("QQ_LOG", "1")
        pb.evaluate(W.random_params(1, 2, 505), grad=True)
        with pytest.raises(N.QQError):
            pb.evaluate(np.array([[0.1, np.nan]]))
        monkeypatch.delenv("QQ_LOG")
        err = capfd.readouterr().err
        assert "[qq] qq_evaluate n=8 p=1 batch=2 flags=0x3 status=0" in err
        assert "status=-1" in err and "not finite" in err
    finally:
        pb.close()
        os.environ.pop("QQ_LOG", None)


def test_poisoned_static_workspace_changes_nothing(monkeypatch):
    """The allocation-free entry point under QQ_POISON: its fixed array is filled with NaN words before
    each call's kernels, and the results still equal the unpoisoned qq_evaluate ones bit for bit."""
    inst = W.dense_gaussian_upper(16, 506)
    pb = Problem(inst.H, inst.f, inst.c0)
    try:
        x = W.random_params(2, 3, 507)
        e_r, g_r = pb.evaluate(x, grad=True)
        monkeypatch.setenv("QQ_POISON", "1")
        e, g = np.empty(3), np.empty((3, 4))
        N.qq_evaluate_static(pb.handle, 2, 3, x, N.QQ_ENERGY | N.QQ_GRAD, None, e, g)
        assert np.array_equal(e, e_r) and np.array_equal(g, g_r)
    finally:
        pb.close()
