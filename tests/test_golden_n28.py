"""The stored FP64 oracle results for the n = 28, p = 8 benchmark workload (CPU only).

tests/golden/regular3_n28_p8_oracle.json is written by tests/golden/make_regular3_n28_oracle.py,
which calls only the oracle and the seeded input generators.  These checks pin that the stored
values still belong to the inputs the generators draw today (SHA-256 of the instance and of each
angle vector) and that they are well formed: 2p finite gradient entries per start and an energy
within the bound |C(z)| <= |c0| + sum |l_i| + sum |b_ij| of the canonical form (eq. (4)-(6)).
The GPU comparison is in test_gpu_fullsize.py.
"""
import json
import os

import numpy as np

from oracle import oracle as O
from paper_2606_26297_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "regular3_n28_p8_oracle.json")


def digest(*arrays):
    import hashlib

    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a, dtype=np.float64).tobytes())
    return h.hexdigest()


def test_stored_oracle_values_match_the_generators():
    ref = json.load(open(GOLDEN))
    inst, x = W.workload3()
    assert ref["n"] == inst.n == 28 and ref["p"] == 8
    assert ref["instance_sha256"] == digest(inst.H, inst.f, np.array([inst.c0]))
    assert len(ref["diagonal_sha256"]) == 64 and int(ref["diagonal_sha256"], 16) >= 0
    ell, b = O.canonicalise(inst.H, inst.f)
    bound = abs(inst.c0) + np.sum(np.abs(ell)) + np.sum(np.abs(b))
    assert [s["start"] for s in ref["starts"]] == [0, 1]
    for s in ref["starts"]:
        assert s["x_sha256"] == digest(x[s["start"]])
        g = np.array(s["gradient"])
        assert g.shape == (16,) and np.all(np.isfinite(g)) and np.isfinite(s["energy"])
        assert abs(s["energy"]) <= bound
