"""Writes uneven512_oracle.json: the FP64 CPU oracle's energy J(x) (eq. (17)) and adjoint gradient
for every one of the 512 problems of the uneven batch (paper_2606_26297_amd.workloads.workload4:
dense symmetric integer QUBOs, n ~ U{10..22}, p ~ U{1..6}, one angle set U[0, pi] each, seeds
104 / 204).

Calls only the oracle (cost diagonal, state by eq. (10)-(13), energy, adjoint gradient) and the
seeded input generators; nothing here touches the GPU library.  The problems are spread over worker
processes (about 8 minutes of single-core work in all).  The file records a SHA-256 digest of each
problem's (H, f, c0) and angle vector, so a test can check that the generators still draw the same
inputs, and the single-core seconds each problem took.

    python tests/golden/make_uneven512_oracle.py [--workers 8]
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

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "uneven512_oracle.json")


def digest(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a, dtype=np.float64).tobytes())
    return h.hexdigest()


def one_problem(k):
    inst, x = W.workload4()[k]
    t0 = time.perf_counter()
    d = O.cost_diagonal(inst.H, inst.f, inst.c0)
    e, g = O.gradient(d, x[0])
    return {"k": k, "n": inst.n, "p": x.shape[1] // 2,
            "instance_sha256": digest(inst.H, inst.f, np.array([inst.c0])), "x_sha256": digest(x[0]),
            "energy": float(e), "gradient": [float(v) for v in g],
            "seconds": round(time.perf_counter() - t0, 3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=min(8, os.cpu_count() or 1))
    args = ap.parse_args()
    items = W.workload4()
    # largest problems first, so the pool's tail is short
    order = sorted(range(len(items)), key=lambda k: -(items[k][0].n * 100 + items[k][1].shape[1]))
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(args.workers) as pool:
        res = pool.map(one_problem, order, chunksize=1)
    res.sort(key=lambda r: r["k"])
    out = {
        "what": "FP64 CPU oracle: energy J(x) (eq. (17)) and adjoint gradient (interleaved like x) of every "
                "problem of the uneven batch",
        "workload": "uneven512 (workloads.workload4: 512 dense symmetric integer QUBOs, entries U{-10..10}, "
                    "n ~ U{10..22}, p ~ U{1..6}, seed 104; one angle set U[0, pi] each, seed 204)",
        "count": len(res),
        "single_core_seconds_total": round(sum(r["seconds"] for r in res), 1),
        "problems": res,
        "script": "tests/golden/make_uneven512_oracle.py",
    }
    with open(OUT, "w") as fh:
        json.dump(out, fh, separators=(",", ":"))
        fh.write("\n")
    print(f"{len(res)} problems, {out['single_core_seconds_total']} s single-core, "
          f"{time.perf_counter() - t0:.1f} s wall")


if __name__ == "__main__":
    main()
