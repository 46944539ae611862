"""The stored FP64 oracle results of the uneven batch and of the two small workloads (CPU only).

tests/golden/uneven512_oracle.json and tests/golden/small_workloads_oracle.json are written by the
make_*.py scripts beside them, which call only the oracle and the seeded input generators.  These
checks pin that the stored values still belong to the inputs the generators draw today (SHA-256
digests), that they are the oracle's own results (a few recomputed here and compared exactly), and
that they are well formed (finite, 2p gradient entries, energies inside the range of C, probabilities
ordered).  The GPU comparisons are in test_gpu_many.py, test_gpu_workloads.py and bench.py.
"""
import hashlib
import json
import os

import numpy as np

from oracle import oracle as O
from paper_2606_26297_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def digest(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a, dtype=np.float64).tobytes())
    return h.hexdigest()


def test_uneven512_stored_values_match_generators_and_oracle():
    ref = json.load(open(os.path.join(GOLDEN, "uneven512_oracle.json")))
    items = W.workload4()
    assert ref["count"] == len(ref["problems"]) == len(items) == 512
    for k, ((inst, x), r) in enumerate(zip(items, ref["problems"])):
        assert r["k"] == k and r["n"] == inst.n and r["p"] == x.shape[1] // 2
        assert r["instance_sha256"] == digest(inst.H, inst.f, np.array([inst.c0])), k
        assert r["x_sha256"] == digest(x[0]), k
        g = np.array(r["gradient"])
        assert g.shape == (2 * r["p"],) and np.all(np.isfinite(g)) and np.isfinite(r["energy"])
    # the stored numbers are the oracle's: recompute the smallest problems exactly
    small = sorted(range(len(items)), key=lambda k: (items[k][0].n, k))[:4]
    for k in small:
        inst, x = items[k]
        d = O.cost_diagonal(inst.H, inst.f, inst.c0)
        e, g = O.gradient(d, x[0])
        assert e == ref["problems"][k]["energy"] and list(g) == ref["problems"][k]["gradient"], k
        assert d.min() <= e <= d.max()


def test_small_workloads_stored_values():
    ref = json.load(open(os.path.join(GOLDEN, "small_workloads_oracle.json")))
    inst1, x1 = W.workload1()
    r1 = ref["workload1"]
    assert r1["instance_sha256"] == digest(inst1.H, inst1.f, np.array([inst1.c0])) and r1["x"] == list(x1[0])
    d1 = O.cost_diagonal(inst1.H, inst1.f, inst1.c0)
    assert O.energy(d1, x1[0]) == r1["energy"]
    assert r1["argmin_cost_index"] == O.argmin_cost(d1) and r1["cost_min"] == d1.min()
    P = np.array(r1["top10_probability"])
    assert np.all(np.diff(P) <= 0) and r1["argmax_probability_index"] == r1["top10_index"][0]
    inst2, x2 = W.workload2()
    r2 = ref["workload2"]
    assert r2["instance_sha256"] == digest(inst2.H, inst2.f, np.array([inst2.c0])) and r2["x_sha256"] == digest(x2)
    e2 = np.array(r2["energy"])
    assert e2.shape == (256,) and np.all(np.isfinite(e2))
    d2 = O.cost_diagonal(inst2.H, inst2.f, inst2.c0)
    assert np.all((d2.min() <= e2) & (e2 <= d2.max()))
    assert O.energy(d2, x2[5]) == e2[5]
