"""Allocation strategies (host only, no GPU): the oracle pinned on Fig. 1, and the library's C-ABI
functions against the oracle.

* Fig. 1: on panel (a)'s six-variable graph with two QPUs of three, the graph-aware greedy finds the
  printed graph-aware split {1,4,5} / {2,3,6} with 2 cross terms (remote estimate 4p), the contiguous
  split {1,2,3} / {4,5,6} has 5 under panel (a)'s edges, the printed manual split has 4, and the
  candidate selection picks the graph-aware one;
* balanced capacities by their closed form; validity (every variable once, capacities, every QPU
  used) and the cross counts of the greedy by brute force on random weighted graphs;
* the library's qq_balanced_capacities / qq_allocation / qq_allocation_candidates equal the oracle
  on random dense, sparse and integer instances (bit-exact: integer outputs).
"""
import json
import os

import numpy as np
import pytest

from oracle import allocation as A
from paper_2606_26297_amd import native as N
from paper_2606_26297_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def fig1():
    with open(os.path.join(GOLDEN, "fig1_allocation.json")) as fh:
        g = json.load(fh)
    H = np.zeros((6, 6))
    for i, j in g["panel_a_edges"]:
        H[min(i, j) - 1, max(i, j) - 1] = 1.0
    return g, H


def as_sets(q):
    return sorted(sorted(int(i) + 1 for i in np.flatnonzero(np.asarray(q) == m)) for m in set(q))


def test_fig1_graph_aware_contiguous_manual():
    g, H = fig1()
    al = g["allocations"]
    q = A.graph_aware(H, [3, 3])
    assert as_sets(q) == sorted([al["graph_aware"]["qpu1"], al["graph_aware"]["qpu2"]])
    assert A.cross_count(H, q) == al["graph_aware"]["printed_cross"] == 2
    qc = A.contiguous(6, [3, 3])
    assert as_sets(qc) == [al["contiguous"]["qpu1"], al["contiguous"]["qpu2"]]
    assert A.cross_count(H, qc) == al["contiguous"]["cross_from_panel_a_edges"] == 5
    manual = [0 if v in al["manual"]["qpu1"] else 1 for v in range(1, 7)]
    cands, cross, remote, best = A.candidates(H, 2, 3, [3, 3], manual)
    assert cross == [2, 5, al["manual"]["printed_cross"]] and remote == [12, 30, 24] and best == 0


def test_balanced_capacities_closed_form():
    assert A.balanced_capacities(7, 3) == [3, 2, 2]
    assert A.balanced_capacities(32, 4) == [8, 8, 8, 8]
    assert A.balanced_capacities(5, 5) == [1] * 5


def brute_cross(H, q):
    n = H.shape[0]
    return sum(1 for i in range(n) for j in range(i + 1, n) if (H[i, j] + H[j, i]) != 0 and q[i] != q[j])


@pytest.mark.parametrize("seed", range(6))
def test_greedy_allocations_are_valid(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(4, 20))
    M = int(rng.integers(1, min(n, 6) + 1))
    H = np.triu(rng.normal(size=(n, n)) * (rng.uniform(size=(n, n)) < 0.4), 1)
    caps = A.balanced_capacities(n, M)
    caps[0] += int(rng.integers(0, 3))  # spare room on one QPU
    for q in (A.graph_aware(H, caps), A.contiguous(n, caps)):
        cnt = np.bincount(q, minlength=M)
        assert len(q) == n and np.all(cnt >= 1) and np.all(cnt <= caps)
        assert A.cross_count(H, q) == brute_cross(H, q)


CASES = [("gauss_n12_M3", lambda: W.dense_gaussian_upper(12, 81).H, 3),
         ("reg_n20_M4", lambda: W.regular_graph_qubo(20, 82).H, 4),
         ("int_n16_M2", lambda: W.dense_integer_symmetric(16, 83).H, 2),
         ("reg_n28_M5", lambda: W.regular_graph_qubo(28, 84).H, 5),
         ("multi_qpu_n32_M4", lambda: W.workload5()[0].H, 4)]


@pytest.mark.parametrize("name,maker,M", CASES, ids=[c[0] for c in CASES])
def test_library_allocation_equals_oracle(name, maker, M):
    H = maker()
    n = H.shape[0]
    assert list(N.qq_balanced_capacities(n, M)) == A.balanced_capacities(n, M)
    for strategy, ref in ((N.QQ_ALLOC_GRAPH, A.graph_aware(H, A.balanced_capacities(n, M))),
                          (N.QQ_ALLOC_CONTIGUOUS, A.contiguous(n, A.balanced_capacities(n, M)))):
        q, x = N.qq_allocation(H, M, strategy=strategy)
        assert list(q) == ref and x == A.cross_count(H, ref)
    manual = [i % M for i in range(n)]
    q, cross, remote, best = N.qq_allocation_candidates(H, M, 3, manual=manual)
    rq, rc, rr, rb = A.candidates(H, M, 3, None, manual)
    assert [list(v) for v in q] == rq and list(cross) == rc and list(remote) == rr and best == rb


def test_allocation_validation():
    _, H = fig1()
    for args in ((H, 0), (H, 7), (H, 2, [2, 3]), (H, 2, [0, 6])):
        with pytest.raises(N.QQError) as ei:
            N.qq_allocation(*args)
        assert ei.value.status == N.QQ_E_INVALID
    with pytest.raises(N.QQError):
        N.qq_allocation(H, 2, strategy=7)
    with pytest.raises(N.QQError):
        N.qq_allocation_candidates(H, 2, 3, manual=[0, 0, 0, 0, 0, 0])  # QPU 1 unused
    with pytest.raises(N.QQError):
        N.qq_allocation_candidates(H, 2, 0)
