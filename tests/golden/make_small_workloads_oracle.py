"""Writes small_workloads_oracle.json: FP64 CPU oracle results for two paper-shaped workloads.

  * the 12-variable dense integer case (workloads.workload1: entries U{-10..10}, seed 101, p = 1,
    (gamma, beta) = (0.4, 0.7)): the energy J(x) (eq. (17)), the most probable basis index and the
    lowest-cost basis index (ties to the lower index), the top-10 (index, probability) list, and the
    single-core seconds of one energy evaluation;
  * the unit-commitment-shaped case (workloads.workload2: 20 units, seed 102; p = 4, 256 angle sets
    U[0, pi], seed 202): the energy of every set and the single-core seconds of each evaluation.

Calls only the oracle (cost diagonal, state by eq. (10)-(13), energy) and the seeded input
generators; nothing here touches the GPU library.  SHA-256 digests of the inputs let a test check
that the generators still draw the same values.

    python tests/golden/make_small_workloads_oracle.py [--workers 8]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2606_26297_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "small_workloads_oracle.json")


def digest(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a, dtype=np.float64).tobytes())
    return h.hexdigest()


_D2 = None


def uc_energy(b):
    _, x = W.workload2()
    t0 = time.perf_counter()
    e = O.energy(_D2, x[b])
    return b, float(e), time.perf_counter() - t0


def main():
    global _D2
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=min(8, os.cpu_count() or 1))
    args = ap.parse_args()

    inst1, x1 = W.workload1()
    d1 = O.cost_diagonal(inst1.H, inst1.f, inst1.c0)
    t0 = time.perf_counter()
    e1 = O.energy(d1, x1[0])
    t_e1 = time.perf_counter() - t0
    P = O.probabilities(O.qaoa_state(d1, x1[0]))
    top_idx = O.topk(P, 10)
    top_p = P[top_idx]
    w1 = {"workload": "workload1: n = 12 dense symmetric integer QUBO (seed 101), p = 1, (gamma, beta) = (0.4, 0.7)",
          "instance_sha256": digest(inst1.H, inst1.f, np.array([inst1.c0])), "x": [float(v) for v in x1[0]],
          "energy": float(e1), "argmax_probability_index": int(top_idx[0]),
          "argmin_cost_index": int(O.argmin_cost(d1)), "cost_min": float(np.min(d1)),
          "top10_index": [int(v) for v in top_idx], "top10_probability": [float(v) for v in top_p],
          "seconds_energy": round(t_e1, 6)}

    inst2, x2 = W.workload2()
    _D2 = O.cost_diagonal(inst2.H, inst2.f, inst2.c0)
    with mp.get_context("fork").Pool(args.workers) as pool:
        res = sorted(pool.map(uc_energy, range(x2.shape[0])))
    w2 = {"workload": "workload2: unit-commitment-shaped QUBO, 20 units (seed 102), p = 4, 256 angle sets "
                      "U[0, pi] (seed 202)",
          "instance_sha256": digest(inst2.H, inst2.f, np.array([inst2.c0])), "x_sha256": digest(x2),
          "energy": [e for _, e, _ in res], "seconds_per_energy": [round(s, 4) for _, _, s in res]}
    out = {"what": "FP64 CPU oracle results of the 12-variable integer case and the unit-commitment-shaped case",
           "workload1": w1, "workload2": w2, "script": "tests/golden/make_small_workloads_oracle.py"}
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(f"workload1 E = {e1:.12g}; workload2: {len(res)} energies, "
          f"{sum(s for _, _, s in res):.1f} s single-core")


if __name__ == "__main__":
    main()
