"""TEST INFRASTRUCTURE -- the oracle of the variable-to-QPU allocation strategies.

Only tests may import this module; the product never does.  It follows the multi-QPU variable
allocation section of the paper (Fig. 1): balanced capacities, the contiguous assignment, a
graph-aware greedy on the weighted coupling graph, candidate allocations with their cross-QPU term
counts and remote-CNOT estimates 2 x cross x p, and selection by the fewest cross terms.  The
paper names the greedy and the tie priority but does not define them; the readings are:

* weights w_ij = |H_ij + H_ji|, strength s(v) = sum_u w_uv;
* QPUs are filled in turn; a QPU starts from the unassigned variable of largest strength and then
  takes the unassigned variable of largest gain 2 w(v, QPU) - s(v) until full, ties to the lower
  index; every QPU leaves one variable for each later QPU and the last takes the rest;
* candidates in the order graph-aware, contiguous, manual; ties in the cross count go to the
  earlier one.
"""
from __future__ import annotations

import numpy as np


def balanced_capacities(n, M):
    return [n // M + (1 if m < n % M else 0) for m in range(M)]


def weights(H):
    H = np.asarray(H, dtype=np.float64)
    W = np.abs(H + H.T)
    np.fill_diagonal(W, 0.0)
    return W


def cross_count(H, q):
    W = weights(H)
    n = W.shape[0]
    return sum(1 for i in range(n) for j in range(i + 1, n) if W[i, j] != 0.0 and q[i] != q[j])


def contiguous(n, caps):
    M = len(caps)
    q, i = [], 0
    for m in range(M):
        room = min(caps[m], n - i - (M - 1 - m))
        q += [m] * room
        i += room
    return q


def graph_aware(H, caps):
    W = weights(H)
    n, M = W.shape[0], len(caps)
    strength = [float(sum(W[v, u] for u in range(n))) for v in range(n)]
    q = [-1] * n
    left = n
    for m in range(M):
        room = left if m == M - 1 else min(caps[m], left - (M - 1 - m))
        members = []
        for k in range(room):
            best, key = None, None
            for v in range(n):
                if q[v] >= 0:
                    continue
                inside = float(sum(W[v, u] for u in members))
                kv = strength[v] if k == 0 else 2.0 * inside - strength[v]
                if best is None or kv > key:
                    best, key = v, kv
            q[best] = m
            members.append(best)
            left -= 1
    return q


def candidates(H, M, p, caps=None, manual=None):
    n = np.asarray(H).shape[0]
    caps = balanced_capacities(n, M) if caps is None else list(caps)
    cands = [graph_aware(H, caps), contiguous(n, caps)]
    if manual is not None:
        cands.append(list(manual))
    cross = [cross_count(H, q) for q in cands]
    best = min(range(len(cands)), key=lambda j: (cross[j], j))
    return cands, cross, [2 * x * p for x in cross], best
