"""Benchmark: batched complex64 QAOA energy + adjoint gradient at n = 28, p = 8.

Workload (one "step"): the 28-node random 3-regular QUBO (edge weights U[0,1],
linear terms N(0, 0.5^2), seeded), p = 8, 64 multi-start parameter sets drawn
U[0, pi]; one step evaluates J(x) and all 16 partial derivatives for every
start through the C ABI (qq_evaluate, QQ_GRAD, device-resident params and
outputs), in waves of `--wave` starts (default 64, all starts in one call: the
widest batch measured fastest per byte on MI355X, 16 -> 32 -> 64 giving 23.0 ->
24.7 -> 25.9 evaluations/s; its 256 GiB of psi and lambda fit the 288 GB HBM).
Inputs are resident in HBM before the
timed region.  Prints one JSON line.

Before timing, the schedule of that evaluation (workgroups per state, pairing of
the high qubit runs) is autotuned through the C ABI (qq_autotune; HIP-event timed
candidates, see "schedule" in the output).

Extra measurements in the same run:
  * per-launch HIP-event timing of every pass kernel during the timed steps
    (roofline of the dominant kernel: algorithmic bytes / launch time vs 8 TB/s),
    with the counter-measured HBM bytes per launch beside the algorithmic ones
    where the committed counter profile was taken on the current kernel sources;
  * the plain complex128 per-gate path (one kernel per gate, one parameter
    set per call) on the same GPU, for the speed-up ratio (one warm-up, median
    of three);
  * parity of the timed results: starts 0-1 against the stored FP64 oracle
    values of this instance, and against the complex128 fused path;
  * the 12-variable integer case (complex128, p = 1) and the unit-commitment-
    shaped batch (n = 20, p = 4, 256 sets, energy only): throughput, and the
    results against stored FP64 oracle values;
  * the CPU oracle (single thread, FP64, pinned to one core) on bounded samples
    of the timed workload (scaled to n = 28, p = 8) and of the other
    workloads, with the host's core count and CPU model;
  * the uneven batch (512 dense integer QUBOs, n in 10..22, p in 1..6, energy +
    gradient): one autotuned persistent launch (qq_evaluate_many) against one
    qq_evaluate call per problem, both with device-resident inputs and outputs,
    and every result against the stored FP64 oracle values;
  * the cost diagonal, min/max, probabilities and top-k kernels on the timed
    instance (one parameter set);
  * the multi-QPU workload at full size (n = 32, 4 QPUs of 8, p = 2, 2 parameter
    sets): monolithic against partitioned (per-QPU local and cross phases)
    energy + gradient, with the cross-coupling count and remote-CNOT estimate.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "QAOA energy+grad evals/s and HBM GB/s at n=28 p=8, <=1e-5 rel vs FP64 oracle"
HBM_PEAK_GBS = 8000.0
KERNEL_SRCS = [os.path.join(ROOT, "paper_2606_26297_amd", "csrc", f)
               for f in ("qq_device.h", "qq_passes.h", "qq_generic.h", "qq_fast.hip", "qq_many.hip", "qq_kernels.hip")]


def kernel_hash() -> str:
    """Hash of the kernel sources; counter-derived traffic is only reported for the source it was taken on."""
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel_name: str):
    """Counter-derived HBM bytes per launch from profiles/, if taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_src_sha256_16") != kernel_hash():
        return None
    entry = t.get("kernels", {}).get(kernel_name)
    return None if entry is None else entry.get("hbm_bytes_per_launch")


GOLDEN = os.path.join(ROOT, "tests", "golden")


def load_golden(name: str):
    """Stored FP64 oracle values (written by the scripts beside them in tests/golden, which call only the
    oracle and the seeded input generators)."""
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


def host_info():
    """Core count, the cores this process may use and the CPU model of the host."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "usable_cores": len(os.sched_getaffinity(0)), "cpu_model": model}


def cpu_baseline():
    """The FP64 oracle (single-threaded C), pinned to one core of this host, on bounded samples:

    * the timed workload's family: one energy + adjoint-gradient evaluation of the 24-node 3-regular
      instance of the same generator at p = 4, scaled to n = 28, p = 8 by 2^4 * (28/24) * (8/4) (work
      grows as n 2^n per layer, linearly in p); the oracle's measured n = 28, p = 8 seconds stored
      with the benchmark instance's oracle values are reported beside it;
    * the 12-variable integer case (p = 1, energy), every 16th set of the unit-commitment-shaped
      batch (n = 20, p = 4, energy) and every 32nd problem of the uneven batch (energy + gradient,
      the cost diagonal included), each scaled to its whole workload where it is a sample.
    """
    import numpy as np

    from oracle import oracle as O
    from paper_2606_26297_amd import workloads as W

    core = min(os.sched_getaffinity(0))
    saved = os.sched_getaffinity(0)
    os.sched_setaffinity(0, {core})
    try:
        inst = W.regular_graph_qubo(24, W.INSTANCE_SEEDS[3])
        d = O.cost_diagonal(inst.H, inst.f, inst.c0)
        x = W.random_params(4, 1, W.PARAM_SEEDS[3])
        t0 = time.perf_counter()
        O.gradient(d, x[0])
        t24 = time.perf_counter() - t0
        del d
        scale = 2.0 ** 4 * (28.0 / 24.0) * (8.0 / 4.0)
        per_eval = t24 * scale

        inst1, x1 = W.workload1()
        d1 = O.cost_diagonal(inst1.H, inst1.f, inst1.c0)
        reps = 50
        t0 = time.perf_counter()
        for _ in range(reps):
            O.energy(d1, x1[0])
        t1 = (time.perf_counter() - t0) / reps

        inst2, x2 = W.workload2()
        d2 = O.cost_diagonal(inst2.H, inst2.f, inst2.c0)
        sel2 = list(range(0, x2.shape[0], 16))
        t0 = time.perf_counter()
        for b in sel2:
            O.energy(d2, x2[b])
        t2 = (time.perf_counter() - t0) / len(sel2)
        del d2

        items = W.workload4()
        sel4 = list(range(0, len(items), 32))
        work = [items[k][0].n * (1 << items[k][0].n) * (items[k][1].shape[1] // 2) for k in range(len(items))]
        t0 = time.perf_counter()
        for k in sel4:
            inst4, x4 = items[k]
            O.gradient(O.cost_diagonal(inst4.H, inst4.f, inst4.c0), x4[0])
        t4 = time.perf_counter() - t0
        t4_all = t4 * sum(work) / sum(work[k] for k in sel4)
    finally:
        os.sched_setaffinity(0, saved)
    stored = load_golden("regular3_n28_p8_oracle.json")
    measured28 = [s["seconds"] for s in stored["starts"]]
    return {"value": 1.0 / per_eval, "unit": "evals/s", "cores": 1, "kind": "oracle",
            "sample": f"one energy+adjoint-gradient evaluation of the 24-node 3-regular instance of the timed "
                      f"workload's generator at p = 4 ({t24:.1f} s, single-threaded FP64 C pinned to core {core}); "
                      f"value extrapolated to n = 28, p = 8 by 2^4*(28/24)*(8/4) = {scale:.2f}",
            "seconds_sample": round(t24, 3), "extrapolated_seconds_per_eval": round(per_eval, 1),
            "measured_n28_p8_seconds_per_eval": measured28,
            "measured_n28_where": "the same oracle on the benchmark instance itself (starts 0 and 1, stored with "
                                  "its values in tests/golden/regular3_n28_p8_oracle.json), timed in the "
                                  "8-core development container, two starts in parallel processes",
            "host": host_info(), "pinned_core": core,
            "configs": {
                "workload1_n12_p1_c128": {"seconds_per_energy": t1, "energies_per_s": 1.0 / t1,
                                          "sample": f"{reps} repetitions of the one evaluation"},
                "workload2_uc_n20_p4": {"seconds_per_energy": round(t2, 4), "energies_per_s": round(1.0 / t2, 3),
                                        "seconds_for_256": round(256 * t2, 1),
                                        "sample": f"{len(sel2)} of the 256 angle sets (every 16th)"},
                "workload4_uneven512": {"seconds_sample": round(t4, 2), "problems_sample": len(sel4),
                                        "extrapolated_seconds_for_512": round(t4_all, 1),
                                        "problems_per_s": round(len(items) / t4_all, 3),
                                        "sample": f"every 32nd problem ({len(sel4)}), energy + adjoint gradient "
                                                  "with the cost diagonal; scaled by the work sum n 2^n p",
                                        "stored_single_core_seconds_for_512": load_golden(
                                            "uneven512_oracle.json")["single_core_seconds_total"]},
            }}


def oracle_multicore_uneven(max_workers=15, every=4):
    """The oracle on every `every`-th problem of the uneven batch (energy + adjoint gradient with the cost
    diagonal), spread over independent forked processes, one per core (each pinned to its own core, the
    problems split by the work estimate n 2^n p, largest first): the oracle's throughput on C cores.
    Runs before this process touches the GPU, so the children hold no device state."""
    import multiprocessing as mp

    from oracle import oracle as O
    from paper_2606_26297_amd import workloads as W

    cores = sorted(os.sched_getaffinity(0))[:max_workers]
    items = W.workload4()
    sel = list(range(0, len(items), every))
    work = {k: items[k][0].n * (1 << items[k][0].n) * (items[k][1].shape[1] // 2) for k in range(len(items))}
    parts = [[] for _ in cores]
    loads = [0.0] * len(cores)
    for k in sorted(sel, key=lambda k: -work[k]):
        j = loads.index(min(loads))
        parts[j].append(k)
        loads[j] += work[k]

    def run(core, ks):
        os.sched_setaffinity(0, {core})
        for k in ks:
            inst, x = items[k]
            O.gradient(O.cost_diagonal(inst.H, inst.f, inst.c0), x[0])

    ctx = mp.get_context("fork")
    procs = [ctx.Process(target=run, args=(c, ks)) for c, ks in zip(cores, parts) if ks]
    t0 = time.perf_counter()
    for pr in procs:
        pr.start()
    for pr in procs:
        pr.join()
    wall = time.perf_counter() - t0
    ok = all(pr.exitcode == 0 for pr in procs)
    scale = sum(work.values()) / sum(work[k] for k in sel)
    return {"cores": len(procs), "problems_sample": len(sel), "seconds_sample": round(wall, 2),
            "extrapolated_seconds_for_512": round(wall * scale, 1), "problems_per_s": round(len(sel) / wall, 3),
            "all_workers_ok": ok,
            "sample": f"every {every}th problem ({len(sel)}), one forked process per core, each pinned, the "
                      "problems split by the work estimate n 2^n p; scaled to 512 by the work sum"}


def progress(msg):
    """Stage lines on stderr (stdout carries only the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def guarded_leg(items, pbs, opt, ref):
    """The guarded evaluation of the uneven batch (host inputs and outputs): complex64 persistent launch, then
    complex128 for the sets whose stated complex64 gradient bound exceeds 1e-5 of the gradient."""
    import numpy as np

    import torch

    from paper_2606_26297_amd import native as N
    from paper_2606_26297_amd.qaoa import evaluate_many_guarded

    xs_h = [x for _, x in items]
    evaluate_many_guarded(pbs, xs_h, tol=1e-5, options=opt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    eg, gg, up, errb = evaluate_many_guarded(pbs, xs_h, tol=1e-5, options=opt)
    t_guard = time.perf_counter() - t0
    gq = [float(np.max(np.abs(gg[k][0] - np.array(ref[k]["gradient"]))) / np.max(np.abs(ref[k]["gradient"])))
          for k in range(len(items))]
    guarded = {"ms": round(1000 * t_guard, 2), "sets_in_complex128": int(sum(int(u[0]) for u in up)),
               "grad_rel_max": max(gq), "grad_rel_over_1e-5": int(sum(v > 1e-5 for v in gq)),
               "bound_holds": bool(all(gq[k] * np.max(np.abs(ref[k]["gradient"])) <= errb[k][0]
                                       for k in range(len(items)))),
               "note": "host inputs and outputs, workspaces allocated by the library; the flagged sets are "
                       "recomputed by one persistent complex128 launch (qq_evaluate_many with QQ_C128)"}
    # the two launches of a second guarded call, timed with HIP events
    N.qq_profile_enable(True)
    N.qq_profile_read()
    evaluate_many_guarded(pbs, xs_h, tol=1e-5, options=opt)
    N.qq_profile_enable(False)
    recs = [r for r in N.qq_profile_read() if r["kind"] == 4]
    guarded["kernel_ms"] = {N.kernel_name(r): round(r["ms"], 3) for r in recs}
    guarded["kernel_algorithmic_GBps"] = {N.kernel_name(r): round(r["bytes"] / (r["ms"] / 1000.0) / 1e9, 1)
                                          for r in recs}
    return guarded


def uneven_batch(dev, reps=5, pinned=None, persistent_only=False, guarded_only=False):
    """The 512-problem uneven batch: persistent launch vs per-problem launches (device-resident).
    pinned: persistent-launch options to use instead of autotuning them; persistent_only: skip the
    per-problem launches (about 26 000 dispatches); guarded_only: only the guarded evaluation."""
    import numpy as np
    import torch

    from paper_2606_26297_amd import native as N
    from paper_2606_26297_amd import workloads as W
    from paper_2606_26297_amd.qaoa import Problem

    items = W.workload4()
    pbs = [Problem(i.H, i.f, i.c0, device=0) for i, _ in items]
    handles = [pb.handle for pb in pbs]
    ps = [x.shape[1] // 2 for _, x in items]
    bs = [x.shape[0] for _, x in items]
    flags = N.QQ_ENERGY | N.QQ_GRAD | N.QQ_PARAMS_ON_DEVICE | N.QQ_OUT_ON_DEVICE
    xs = [torch.tensor(x, device=dev) for _, x in items]
    es = [torch.empty(b, dtype=torch.float64, device=dev) for b in bs]
    gs = [torch.empty(x.shape, dtype=torch.float64, device=dev) for x in xs]
    stream = torch.cuda.current_stream(dev)
    if guarded_only:
        return {"workload": "512 dense integer QUBOs, n ~ U{10..22}, p ~ U{1..6}, 1 parameter set each, energy+grad",
                "guarded": guarded_leg(items, pbs, pinned, load_golden("uneven512_oracle.json")["problems"])}
    if pinned is None:
        opt, tune_ms = N.qq_autotune_many(handles, ps, bs, flags, None, stream)
    else:
        opt, tune_ms = dict(pinned), None
    ws_bytes = N.qq_workspace_size_many(handles, ps, bs, flags, opt)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)

    def many():
        N.qq_evaluate_many(handles, ps, bs, xs, flags, opt, ws, ws_bytes, stream, es, gs)

    many()
    torch.cuda.synchronize()
    N.qq_profile_enable(True)
    N.qq_profile_read()
    t0 = time.perf_counter()
    for _ in range(reps):
        many()
    torch.cuda.synchronize()
    t_many = (time.perf_counter() - t0) / reps
    N.qq_profile_enable(False)
    recs = N.qq_profile_read()
    k_ms = sum(r["ms"] for r in recs) / reps
    k_bytes = sum(r["bytes"] for r in recs) / reps
    e_many = [e.clone() for e in es]
    g_many = [g.clone() for g in gs]
    del ws
    if persistent_only:
        return {"workload": "512 dense integer QUBOs, n ~ U{10..22}, p ~ U{1..6}, 1 parameter set each, energy+grad",
                "persistent_ms": round(1000 * t_many, 3), "persistent_kernel_ms": round(k_ms, 3),
                "persistent_algorithmic_GBps": round(k_bytes / (k_ms / 1000.0) / 1e9, 1), "options": opt}
    wsz = max(N.qq_workspace_size(h, p, b, flags) for h, p, b in zip(handles, ps, bs))
    ws1 = torch.empty(wsz, dtype=torch.uint8, device=dev)

    def per_problem():
        for h, p, b, x, e, g in zip(handles, ps, bs, xs, es, gs):
            N.qq_evaluate(h, p, b, x, flags, ws1, wsz, stream, e, g)

    per_problem()
    torch.cuda.synchronize()
    N.qq_profile_enable(True)
    N.qq_profile_read()
    t0 = time.perf_counter()
    for _ in range(reps):
        per_problem()
    torch.cuda.synchronize()
    t_per = (time.perf_counter() - t0) / reps
    N.qq_profile_enable(False)
    launches = len(N.qq_profile_read()) // reps
    sig = np.array([pb.info.sigma_c for pb in pbs])
    de = max(float(np.max(np.abs(a.cpu().numpy() - b.cpu().numpy()) / np.maximum(np.abs(b.cpu().numpy()), s)))
             for a, b, s in zip(e_many, es, sig))
    # every result of the persistent launch against the stored FP64 oracle values
    ref = load_golden("uneven512_oracle.json")["problems"]
    e_rel, g_rel, g_abs = [], [], []
    for k in range(len(items)):
        gr = np.array(ref[k]["gradient"])
        e_rel.append(abs(float(e_many[k][0]) - ref[k]["energy"]) / max(abs(ref[k]["energy"]), sig[k]))
        dg = float(np.max(np.abs(g_many[k][0].cpu().numpy() - gr)))
        g_rel.append(dg / float(np.max(np.abs(gr))))
        g_abs.append(dg / sig[k])
    guarded = guarded_leg(items, pbs, opt, ref)
    vs_oracle = {"problems": len(items), "energy_rel_max": max(e_rel), "grad_rel_max": max(g_rel),
                 "grad_rel_median": float(np.median(g_rel)), "grad_rel_over_1e-5": int(sum(v > 1e-5 for v in g_rel)),
                 "grad_abs_over_sigma_max": max(g_abs),
                 "metric": "energy |dE|/max(|E|, sigma_C); gradient ||dg||_inf/||g||_inf and ||dg||_inf/sigma_C; "
                           "complex64 states"}
    return {"workload": "512 dense integer QUBOs, n ~ U{10..22}, p ~ U{1..6}, 1 parameter set each, energy+grad",
            "persistent_ms": round(1000 * t_many, 3), "persistent_kernel_ms": round(k_ms, 3),
            "persistent_algorithmic_GBps": round(k_bytes / (k_ms / 1000.0) / 1e9, 1),
            "per_problem_ms": round(1000 * t_per, 3), "per_problem_launches": launches,
            "speedup": round(t_per / t_many, 2), "problems_per_s": round(len(items) / t_many, 1),
            "traffic_bytes_per_launch": load_traffic("many_kernel<%s>" % N.DIAG_TYPE_NAMES[pbs[0].info.diag_bytes]),
            "options": opt, "autotune_best_ms": None if tune_ms is None else round(tune_ms, 3),
            "energy_rel_vs_per_problem": de, "vs_oracle": vs_oracle, "guarded": guarded}


def copy_calibration(dev):
    """A plain copy kernel of known size (4 GiB read, 4 GiB written): its FETCH_SIZE / WRITE_SIZE counters
    calibrate the counter-derived HBM traffic of the other kernels, and its rate is a bandwidth reference."""
    import torch

    nbytes = 4 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 3
    c0.record()
    for _ in range(reps):
        dst.copy_(src)
    c1.record()
    torch.cuda.synchronize()
    cms = c0.elapsed_time(c1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return {"bytes": nbytes, "ms_per_copy": round(cms, 4), "read_plus_write_GBps": round(2 * nbytes / (cms / 1e3) / 1e9, 1),
            "kernel": "torch copy_ of a 4 GiB float32 tensor (device to device)"}


def small_workloads(dev, reps=200):
    """The 12-variable integer case (complex128, p = 1, one angle pair) and the unit-commitment-shaped
    batch (n = 20, p = 4, 256 angle sets, complex64, energy only): throughput with device-resident
    inputs and outputs, and the results against the stored FP64 oracle values."""
    import numpy as np
    import torch

    from paper_2606_26297_amd import native as N
    from paper_2606_26297_amd import workloads as W
    from paper_2606_26297_amd.qaoa import Problem

    ref = load_golden("small_workloads_oracle.json")
    stream = torch.cuda.current_stream(dev)
    out = {}

    # 12-variable case: one energy per call, complex128
    inst, x = W.workload1()
    pb = Problem(inst.H, inst.f, inst.c0, device=0)
    flags = N.QQ_ENERGY | N.QQ_C128 | N.QQ_PARAMS_ON_DEVICE | N.QQ_OUT_ON_DEVICE
    xt = torch.tensor(x, device=dev)
    e = torch.empty(1, dtype=torch.float64, device=dev)
    wsb = pb.workspace_size(1, 1, flags)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    for _ in range(10):
        N.qq_evaluate(pb.handle, 1, 1, xt, flags, ws, wsb, stream, e, None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        N.qq_evaluate(pb.handle, 1, 1, xt, flags, ws, wsb, stream, e, None)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    idx, pr, _ = pb.topk(x[0], k=10, c128=True)
    r1 = ref["workload1"]
    sig = pb.info.sigma_c
    out["workload1_n12_p1_c128"] = {
        "evals_per_s": round(1.0 / dt, 1), "us_per_eval": round(1e6 * dt, 2),
        "energy_rel_vs_oracle": abs(float(e.item()) - r1["energy"]) / max(abs(r1["energy"]), sig),
        "argmax_matches_oracle": int(idx[0]) == r1["argmax_probability_index"],
        "argmin_cost_matches_oracle": int(pb.info.argmin_index) == r1["argmin_cost_index"],
        "top10_probability_max_abs_diff": float(np.max(np.abs(np.asarray(pr) - np.asarray(r1["top10_probability"])))),
        "note": "one evaluation per call, launch-bound at this size"}
    pb.close()

    # unit-commitment-shaped batch: 256 sets in one call, complex64, energy only
    inst, x = W.workload2()
    pb = Problem(inst.H, inst.f, inst.c0, device=0)
    p, B = x.shape[1] // 2, x.shape[0]
    flags = N.QQ_ENERGY | N.QQ_PARAMS_ON_DEVICE | N.QQ_OUT_ON_DEVICE
    xt = torch.tensor(x, device=dev)
    e = torch.empty(B, dtype=torch.float64, device=dev)
    wsb = pb.workspace_size(p, B, flags)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    N.qq_evaluate(pb.handle, p, B, xt, flags, ws, wsb, stream, e, None)
    torch.cuda.synchronize()
    N.qq_profile_enable(True)
    N.qq_profile_read()
    k = 5
    t0 = time.perf_counter()
    for _ in range(k):
        N.qq_evaluate(pb.handle, p, B, xt, flags, ws, wsb, stream, e, None)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / k
    N.qq_profile_enable(False)
    recs = N.qq_profile_read()
    by = sum(r["bytes"] for r in recs) / k
    ms = sum(r["ms"] for r in recs) / k
    sig = pb.info.sigma_c
    er = np.array(ref["workload2"]["energy"])
    eh = e.cpu().numpy()
    out["workload2_uc_n20_p4_b256"] = {
        "evals_per_s": round(B / dt, 1), "ms_per_batch": round(1000 * dt, 3),
        "algorithmic_GBps": round(by / (ms / 1000.0) / 1e9, 1), "launches_per_batch": len(recs) // k,
        "energy_rel_vs_oracle_max": float(np.max(np.abs(eh - er) / np.maximum(np.abs(er), sig))),
        "note": "256 states of 8 MiB (2 GiB in all): HBM-resident; energy only"}
    pb.close()
    return out


def aux_kernels(dev, inst, x):
    """Cost diagonal, min/max, probabilities and top-k on the timed instance (one parameter set)."""
    import torch

    from paper_2606_26297_amd import native as N
    from paper_2606_26297_amd.qaoa import Problem

    # one creation first, so the timed one does not include the first touch of fresh device pages
    Problem(inst.H, inst.f, inst.c0, device=0).close()
    N.qq_profile_enable(True)
    N.qq_profile_read()
    pb = Problem(inst.H, inst.f, inst.c0, device=0)
    torch.cuda.synchronize()
    p = x.shape[1] // 2
    flags = N.QQ_PARAMS_ON_DEVICE | N.QQ_OUT_ON_DEVICE
    xt = torch.tensor(x[0], device=dev)
    prob = torch.empty(1 << pb.n, dtype=torch.float64, device=dev)
    N.qq_probabilities(pb.handle, p, xt, flags, prob)
    idx, pr, cost = N.qq_topk(pb.handle, p, xt, N.QQ_PARAMS_ON_DEVICE, 10)
    torch.cuda.synchronize()
    N.qq_profile_enable(False)
    recs = N.qq_profile_read()
    out = {}
    for r in recs:
        if r["kind"] < 5:
            continue
        k = N.kernel_name(r)
        out[k] = {"ms": round(r["ms"], 4), "algorithmic_GBps": round(r["bytes"] / (r["ms"] / 1000.0) / 1e9, 1),
                  "bytes": r["bytes"]}
    out["top1"] = {"index": int(idx[0]), "probability": float(pr[0]), "cost": float(cost[0]),
                   "probability_sum": float(prob.sum())}
    del prob
    pb.close()
    return out


def optimizer(dev, n=22, p_max=5, iterations=60, random_starts=16, perturbed_starts=15):
    """Depth progression with multi-start search (qq_optimize) on a 3-regular instance of the timed
    workload's generator: every depth runs all its starts as one batch of graph-captured Adam steps."""
    import numpy as np
    import torch

    from paper_2606_26297_amd import native as N
    from paper_2606_26297_amd import workloads as W
    from paper_2606_26297_amd.qaoa import Problem

    inst = W.regular_graph_qubo(n, 303)
    pb = Problem(inst.H, inst.f, inst.c0, device=0)
    pts, off = W.optimizer_draws(p_max, random_starts, perturbed_starts, 304)
    opts = {"p_max": p_max, "iterations": iterations, "random_starts": random_starts,
            "perturbed_starts": perturbed_starts, "include_warm": 1, "adam": (0.05, 0.9, 0.999, 1e-8)}
    N.qq_optimize(pb.handle, dict(opts, p_max=1, iterations=2), pts[:2 * random_starts])  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = N.qq_optimize(pb.handle, opts, pts, off)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    info = pb.info
    out = {"workload": f"3-regular graph QUBO, n = {n}, depths 1..{p_max}, {iterations} Adam steps per start, "
                       f"{random_starts} random + 1 warm + {perturbed_starts} perturbed starts per depth "
                       "(depth 1: random only), complex64 energy + adjoint gradient",
           "seconds": round(dt, 3), "adam_steps": int(r["steps"]), "evaluations": int(r["evaluations"]),
           "start_steps_per_s": round(r["steps"] / dt, 1), "best_depth": r["best_depth"],
           "best_start": r["best_start"], "best_energy": r["best_energy"],
           "depth_energy": [float(v) for v in r["depth_energy"]], "cmin": info.cmin, "cmax": info.cmax,
           "approximation_ratio": (info.cmax - r["best_energy"]) / (info.cmax - info.cmin)}
    pb.close()
    return out


def sampling(dev, shots=1_000_000):
    """Shots from the exact distribution of the timed workload's first parameter set (n = 28, p = 8)
    and their metrics."""
    import numpy as np
    import torch

    from paper_2606_26297_amd import native as N
    from paper_2606_26297_amd import workloads as W
    from paper_2606_26297_amd.qaoa import Problem

    inst, x = W.workload3(batch=1)
    pb = Problem(inst.H, inst.f, inst.c0, device=0)
    u = np.random.default_rng(305).uniform(0.0, 1.0, size=shots)
    pb.sample(x[0], u[:1000])  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    z = pb.sample(x[0], u)
    t1 = time.perf_counter()
    info = pb.info
    st = pb.sample_stats(z, margin=0.5, k=10)
    t2 = time.perf_counter()
    out = {"workload": f"regular3_n28_p8 start 0, {shots} shots (state preparation included)",
           "ms_sample": round(1000 * (t1 - t0), 2), "shots_per_s": round(shots / (t1 - t0), 1),
           "ms_stats": round(1000 * (t2 - t1), 2),
           "best_cost": st["best_cost"], "best_cost_mass": st["best_cost_mass"], "low_cost_mass_0.5": st["low_cost_mass"],
           "mean_cost": st["mean_cost"], "distinct": st["distinct"], "exact_cost": info.cmin,
           "exact_cost_mass": st["exact_cost_mass"], "elite_top3": [int(v) for v in st["elite_index"][:3]]}
    pb.close()
    return out


def telegate(dev):
    """One gate-level trajectory of the distributed circuit with explicit TeleGate remote CNOTs: the
    12-variable integer case, 3 QPUs of 4 (contiguous), p = 2, against the exact state."""
    import numpy as np
    import torch

    from paper_2606_26297_amd import native as N
    from paper_2606_26297_amd import workloads as W
    from paper_2606_26297_amd.qaoa import Problem

    inst, _ = W.workload1()
    n = inst.H.shape[0]
    pb = Problem(inst.H, inst.f, inst.c0, device=0)
    cross, _ = pb.set_allocation(W.contiguous_allocation(n, [4, 4, 4]), 3, [4, 4, 4])
    x = W.random_params(2, 1, 306)[0]
    u = np.random.default_rng(307).uniform(size=4 * cross * 2)
    N.qq_telegate_state(pb.handle, n, x, u)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    psi, outcomes, remote = N.qq_telegate_state(pb.handle, n, x, u)
    dt = time.perf_counter() - t0
    exact = pb.state(x, c128=True)
    out = {"workload": f"12-variable integer QUBO, 3 QPUs x 4 (contiguous), p = 2, {cross} cross terms",
           "remote_cnots": int(remote), "measurements": int(outcomes.size), "ms": round(1000 * dt, 2),
           "max_abs_diff_vs_exact_state": float(np.max(np.abs(psi - exact)))}
    pb.close()
    return out


def multi_qpu(dev):
    """The n = 32 multi-QPU workload: monolithic vs partitioned energy + gradient (device-resident)."""
    import numpy as np
    import torch

    from paper_2606_26297_amd import native as N
    from paper_2606_26297_amd import workloads as W
    from paper_2606_26297_amd.qaoa import Problem

    inst, x, alloc = W.workload5()
    n, p, B = inst.H.shape[0], x.shape[1] // 2, x.shape[0]
    Problem(inst.H, inst.f, inst.c0, device=0).close()  # first touch of the 32 GiB outside the timing
    N.qq_profile_enable(True)
    N.qq_profile_read()
    pb = Problem(inst.H, inst.f, inst.c0, device=0)
    torch.cuda.synchronize()
    diag_recs = [r for r in N.qq_profile_read() if r["kind"] == 5]
    N.qq_profile_enable(False)
    caps = [int(c) for c in np.bincount(alloc)]
    cross, remote = pb.set_allocation(alloc, len(caps), caps)
    xt = torch.tensor(x, device=dev)
    out = {"workload": f"dense N(0,1) upper-triangular QUBO, n = {n}, p = {p}, {B} parameter sets, "
                       f"{len(caps)} QPUs x {caps[0]} (contiguous), complex64 energy+grad",
           "cross_terms": cross, "remote_cx_per_layer": remote, "remote_cx_circuit": remote * p}
    if diag_recs:
        r = diag_recs[0]
        out["cost_diag_kernel"] = {"ms": round(r["ms"], 3), "written_GBps": round(r["bytes"] / (r["ms"] / 1e3) / 1e9, 1),
                                   "entries": 1 << n, "terms_per_entry": n + int(np.count_nonzero(np.triu(inst.H, 1))),
                                   "note": "FP64 entries in the canonical summation order, once per problem"}
    res = {}
    for name, part in (("monolithic", False), ("partitioned", True)):
        pb.evaluate(xt, grad=True, partitioned=part)
        torch.cuda.synchronize()
        N.qq_profile_enable(True)
        N.qq_profile_read()
        t0 = time.perf_counter()
        e, g = pb.evaluate(xt, grad=True, partitioned=part)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        N.qq_profile_enable(False)
        recs = N.qq_profile_read()
        by = sum(r["bytes"] for r in recs)
        ms = sum(r["ms"] for r in recs)
        res[name] = (e.cpu().numpy(), g.cpu().numpy())
        out[name] = {"ms": round(1000 * dt, 2), "algorithmic_GBps": round(by / (ms / 1000.0) / 1e9, 1),
                     "launches": len(recs)}
    sig = pb.info.sigma_c
    (e0, g0), (e1, g1) = res["monolithic"], res["partitioned"]
    out["partitioned_overhead"] = round(out["partitioned"]["ms"] / out["monolithic"]["ms"], 3)
    t0 = time.perf_counter()
    _, cross, remote, best = N.qq_allocation_candidates(inst.H, len(caps), p, capacities=caps)
    out["allocation_candidates"] = {"graph_aware_cross": int(cross[0]), "contiguous_cross": int(cross[1]),
                                    "best": ["graph_aware", "contiguous"][best],
                                    "ms": round(1000 * (time.perf_counter() - t0), 3)}
    out["partitioned_vs_monolithic"] = {
        "energy_rel": float(np.max(np.abs(e1 - e0) / np.maximum(np.abs(e0), sig))),
        "grad_rel": float(np.max(np.abs(g1 - g0)) / np.max(np.abs(g0)))}
    pb.close()
    return out


def _short_kernel_name(name: str) -> str:
    """rocprofv3's demangled kernel name without the return type, namespaces and parameter list."""
    name = name.strip()
    if name.startswith("void "):
        name = name[5:]
    name = name.replace("qq::(anonymous namespace)::", "").replace("qq::", "")
    depth = 0
    for i, ch in enumerate(name):  # cut at the parameter list: the first '(' outside template brackets
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0 and i > 0:
            return name[:i]
    return name


def _csv_rows(directory: str, suffix: str):
    import csv
    import glob

    rows = []
    for path in sorted(glob.glob(os.path.join(directory, "**", f"*{suffix}"), recursive=True)):
        with open(path, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    if not rows:
        raise SystemExit(f"no *{suffix} under {directory}")
    return rows


def summarize_counters(workload, stats_dir, fetch_dir, write_dir, command, only=None):
    """Summaries of three rocprofv3 runs of one command: kernel statistics (--kernel-trace --stats) and the
    FETCH_SIZE and WRITE_SIZE counters (KiB per dispatch), each calibrated by a 4 GiB reference copy
    (its counter reading against the 4 GiB it moves).  Per-launch figures use only the dispatches of each
    kernel with its most frequent grid size (the timed configuration); the others are listed apart."""
    from collections import Counter, defaultdict

    stats = _csv_rows(stats_dir, "kernel_stats.csv")
    lines = [f"# rocprofv3 kernel statistics: {workload}", "",
             "Command (on the MI355X box, repository at /root/repo):", "",
             "    cd /tmp && export TMPDIR=/tmp",
             f"    rocprofv3 --kernel-trace --stats -f csv -d <out>/stats -o run -- {command}", "",
             "| kernel | calls | avg ms | min ms | max ms | share % |", "|---|---:|---:|---:|---:|---:|"]
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"])):
        lines.append(f"| `{_short_kernel_name(r['Name'])[:70]}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.3f} | "
                     f"{float(r['MinNs']) / 1e6:.3f} | {float(r['MaxNs']) / 1e6:.3f} | "
                     f"{float(r['Percentage']):.2f} |")
    with open(os.path.join(ROOT, "profiles", f"{workload}_stats.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")

    def per_kernel(directory, counter):
        rows = [r for r in _csv_rows(directory, "counter_collection.csv") if r["Counter_Name"].startswith(counter)]
        by = defaultdict(list)
        for r in rows:
            by[(_short_kernel_name(r["Kernel_Name"]), int(r["Grid_Size"]))].append(float(r["Counter_Value"]) * 1024.0)
        copies = [v for (k, g), vs in by.items() if "copyBuffer" in k for v in vs]
        return by, max(copies) if copies else None

    fetch, f_copy = per_kernel(fetch_dir, "FETCH_SIZE")
    write, w_copy = per_kernel(write_dir, "WRITE_SIZE")
    ref = 4.0 * 2 ** 30
    f_scale = ref / f_copy if f_copy else 1.0
    w_scale = ref / w_copy if w_copy else 1.0
    names = sorted({k for k, _ in fetch} | {k for k, _ in write})
    grid_count = Counter()
    for (k, g), vs in list(fetch.items()) + list(write.items()):
        grid_count[(k, g)] += len(vs)
    path = os.path.join(ROOT, "profiles", "traffic.json")
    traffic = {"kernel_src_sha256_16": kernel_hash(), "workloads": {}, "kernels": {}}
    if os.path.exists(path):
        with open(path) as fh:
            old = json.load(fh)
        if old.get("kernel_src_sha256_16") == traffic["kernel_src_sha256_16"]:
            traffic = old
            traffic.setdefault("workloads", {})
    traffic["workloads"][workload] = command
    tl = [f"# rocprofv3 HBM traffic counters: {workload}", "",
          "Two counter runs (one counter per run) of the same command:", "",
          "    cd /tmp && export TMPDIR=/tmp",
          f"    timeout -s KILL 600 rocprofv3 --pmc FETCH_SIZE -f csv -d <out>/fetch -o run -- {command}",
          f"    timeout -s KILL 600 rocprofv3 --pmc WRITE_SIZE -f csv -d <out>/write -o run -- {command}", "",
          f"Calibration: the 4 GiB reference copy reads FETCH_SIZE = {f_copy / 2 ** 30 if f_copy else float('nan'):.3f} GiB "
          f"and WRITE_SIZE = {w_copy / 2 ** 30 if w_copy else float('nan'):.3f} GiB, so fetch counters are scaled by "
          f"{f_scale:.3f} and write counters by {w_scale:.3f}.  Per-launch rows use each kernel's dispatches of its "
          "most frequent grid size (the timed configuration).", "",
          "| kernel | grid (work-items) | launches | fetch GiB/launch | write GiB/launch | HBM GiB/launch |",
          "|---|---:|---:|---:|---:|---:|"]
    import re

    for k in names:
        if "copyBuffer" in k or "fillBuffer" in k or (only and not re.search(only, k)):
            continue
        grids = [g for (kk, g) in grid_count if kk == k]
        g = max(grids, key=lambda gg: (grid_count[(k, gg)], gg))
        fv, wv = fetch.get((k, g), []), write.get((k, g), [])
        if not fv or not wv:
            continue
        fb = sum(fv) / len(fv) * f_scale
        wb = sum(wv) / len(wv) * w_scale
        traffic["kernels"][k] = {"hbm_bytes_per_launch": fb + wb, "fetch_bytes": fb, "write_bytes": wb,
                                 "grid_size": g, "launches": len(fv), "workload": workload}
        others = sum(len(vs) for (kk, gg), vs in fetch.items() if kk == k and gg != g)
        note = f" (+{others} launches of other sizes)" if others else ""
        tl.append(f"| `{k}`{note} | {g} | {len(fv)} | {fb / 2 ** 30:.2f} | {wb / 2 ** 30:.2f} | {(fb + wb) / 2 ** 30:.2f} |")
    with open(os.path.join(ROOT, "profiles", f"{workload}_traffic.md"), "w") as fh:
        fh.write("\n".join(tl) + "\n")
    with open(path, "w") as fh:
        json.dump(traffic, fh, indent=1)
        fh.write("\n")
    print(f"wrote profiles/{workload}_stats.md, profiles/{workload}_traffic.md, profiles/traffic.json")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--wave", type=int, default=64, help="starts per qq_evaluate call")
    ap.add_argument("--starts", type=int, default=64)
    ap.add_argument("--n", type=int, default=28)
    ap.add_argument("--p", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="time the built-in default schedule")
    ap.add_argument("--no-uneven", action="store_true", help="skip the uneven-batch measurement")
    ap.add_argument("--uneven-only", action="store_true", help="run only the uneven-batch measurement")
    ap.add_argument("--no-multi-qpu", action="store_true", help="skip the n = 32 multi-QPU measurement")
    ap.add_argument("--no-optimizer", action="store_true", help="skip the depth-progression search measurement")
    ap.add_argument("--no-sampling", action="store_true", help="skip the shot-sampling measurement")
    ap.add_argument("--no-telegate", action="store_true", help="skip the TeleGate trajectory measurement")
    ap.add_argument("--schedule", default=None, metavar="G:PAIRING[:ORDER[:SETORDER]]",
                    help="pin this schedule (workgroups per state, set pairing, tile order, set order) "
                         "instead of autotuning")
    ap.add_argument("--guarded-only", action="store_true",
                    help="with --uneven-only: only the guarded evaluation (complex64 launch, complex128 recomputation)")
    ap.add_argument("--persistent-only", action="store_true",
                    help="with --uneven-only: time only the persistent launch (no per-problem launches)")
    ap.add_argument("--multi-qpu-only", action="store_true",
                    help="run only the n = 32 multi-QPU leg (monolithic and partitioned phases)")
    ap.add_argument("--aux-only", action="store_true",
                    help="run only the cost-diagonal / probabilities / top-k leg on the timed instance")
    ap.add_argument("--no-host-buffers", action="store_true",
                    help="skip the step with host parameters and outputs")
    ap.add_argument("--many-options", default=None, metavar="TILES_PER_CHUNK:MAX_WORKGROUPS",
                    help="pin the persistent-launch options of the uneven batch instead of autotuning them")
    ap.add_argument("--summarize-counters", nargs=5, default=None,
                    metavar=("WORKLOAD", "STATS_DIR", "FETCH_DIR", "WRITE_DIR", "COMMAND"),
                    help="write the profiles/ summaries of three rocprofv3 runs of COMMAND (kernel statistics, "
                         "FETCH_SIZE, WRITE_SIZE) and merge their per-launch HBM bytes into profiles/traffic.json; "
                         "CPU only")
    ap.add_argument("--counter-kernels", default=None, metavar="REGEX",
                    help="with --summarize-counters: record per-launch traffic only for kernels matching REGEX")
    ap.add_argument("--no-aux", action="store_true",
                    help="skip the cost-diagonal / probabilities / top-k leg (one-state launches)")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the 12-variable and unit-commitment-shaped workloads")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 4 GiB device copy (reference kernel for the traffic counters) and "
                         "report its rate in the --uneven-only / --aux-only legs (the full run always does)")
    args = ap.parse_args()

    if args.summarize_counters:
        summarize_counters(*args.summarize_counters, only=args.counter_kernels)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library runs its hot path on a single MI355X "
              "(sharding over several GPUs is not built). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2606_26297_amd import native as N
    from paper_2606_26297_amd import workloads as W
    from paper_2606_26297_amd.qaoa import Problem

    oracle_cores = None
    if not (args.no_cpu_baseline or args.uneven_only or args.aux_only or args.multi_qpu_only):
        progress("oracle on several cores (before the GPU is touched)")
        oracle_cores = oracle_multicore_uneven()

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    pinned_many = None
    if args.many_options:
        tpc, cap = (int(v) for v in args.many_options.split(":"))
        pinned_many = {"tiles_per_chunk": tpc, "max_workgroups": cap, "wait_limit_ms": 0.0}
    if args.uneven_only:
        progress("uneven batch")
        res = {"uneven_batch": uneven_batch(dev, pinned=pinned_many, persistent_only=args.persistent_only,
                                            guarded_only=args.guarded_only)}
        if args.copy_calibration:
            res["copy_calibration"] = copy_calibration(dev)
        print(json.dumps(res), flush=True)
        return
    if args.aux_only:
        progress("cost diagonal, probabilities, top-k")
        inst, x = W.workload3(batch=1, p=args.p, n=args.n)
        res = {"aux": aux_kernels(dev, inst, x)}
        if args.copy_calibration:
            res["copy_calibration"] = copy_calibration(dev)
        print(json.dumps(res), flush=True)
        return
    if args.multi_qpu_only:
        progress("n = 32 multi-QPU workload")
        res = {"multi_qpu": multi_qpu(dev)}
        if args.copy_calibration:
            res["copy_calibration"] = copy_calibration(dev)
        print(json.dumps(res), flush=True)
        return
    inst, x = W.workload3(batch=args.starts, p=args.p, n=args.n)
    pb = Problem(inst.H, inst.f, inst.c0, device=0)
    p, S, B = args.p, args.starts, args.wave
    assert S % B == 0
    flags = N.QQ_ENERGY | N.QQ_GRAD | N.QQ_PARAMS_ON_DEVICE | N.QQ_OUT_ON_DEVICE
    xt = torch.tensor(x, dtype=torch.float64, device=dev)
    e_out = torch.empty(S, dtype=torch.float64, device=dev)
    g_out = torch.empty(S, 2 * p, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)

    if args.schedule:
        fields = [int(v) for v in args.schedule.split(":")]
        G, pairing, order, set_order = (fields + [0, 0, 0])[:4]
        N.qq_set_schedule(pb.handle, p, B, flags, {"workgroups_per_state": G, "set_pairing": pairing,
                                                   "tile_order": order, "set_order": set_order})
    schedule = N.qq_get_schedule(pb.handle, p, B, flags)
    if not args.no_autotune and not args.schedule:
        progress("autotuning the schedule")
        schedule = N.qq_autotune(pb.handle, p, B, flags, None, stream)
        progress(f"schedule {schedule}")
    ws_bytes = pb.workspace_size(p, B, flags)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)

    def step():
        for w in range(S // B):
            N.qq_evaluate(pb.handle, p, B, xt[w * B:(w + 1) * B], flags, ws, ws_bytes, stream,
                          e_out[w * B:(w + 1) * B], g_out[w * B:(w + 1) * B])

    progress(f"warmup x{args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    progress(f"timing {args.steps} steps")
    N.qq_profile_enable(True)
    N.qq_profile_read()  # clear
    # one event between consecutive steps (recorded on the launch stream, read after the timed region)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record(stream)
    for i in range(args.steps):
        step()
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    N.qq_profile_enable(False)
    recs = N.qq_profile_read()
    wall = t1 - t0
    ms_per_step = 1000.0 * wall / args.steps
    value = S * args.steps / wall
    step_ms = [round(evs[i].elapsed_time(evs[i + 1]), 3) for i in range(args.steps)]

    # roofline of the dominant kernel (the instantiation with the largest total time)
    by_kind = {}
    for r in recs:
        k = N.kernel_name(r)
        d = by_kind.setdefault(k, {"ms": 0.0, "bytes": 0.0, "launches": 0})
        d["ms"] += r["ms"]
        d["bytes"] += r["bytes"]
        d["launches"] += 1
    dom = max(by_kind, key=lambda k: by_kind[k]["ms"])
    dk = by_kind[dom]
    achieved = dk["bytes"] / (dk["ms"] / 1000.0) / 1e9
    traffic = load_traffic(dom)
    step_bytes = sum(d["bytes"] for d in by_kind.values()) / args.steps
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
                "launches": dk["launches"], "avg_launch_ms": round(dk["ms"] / dk["launches"], 4),
                "algorithmic_bytes_per_launch": dk["bytes"] / dk["launches"]}
    kernels = {}
    for k, v in by_kind.items():
        alg = v["bytes"] / v["launches"]
        cnt = load_traffic(k)
        kernels[k] = {"launches": v["launches"], "avg_ms": round(v["ms"] / v["launches"], 4),
                      "GBps": round(v["bytes"] / max(v["ms"], 1e-9) / 1e6, 1),
                      "algorithmic_bytes_per_launch": alg,
                      "counter_over_algorithmic": None if cnt is None or alg <= 0 else round(cnt / alg, 4)}

    out = {"metric": METRIC, "value": round(value, 3), "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "c64", "data": "synthetic",
           "config": {"workload": f"regular3_n{args.n}_p{p}_starts{S}", "n": args.n, "p": p, "starts": S,
                      "wave": B, "state": "complex64", "accumulators": "fp64"},
           "schedule": schedule,
           "step_ms_each": step_ms, "step_ms_median": round(float(np.median(step_ms)), 3),
           "hbm_GBps_step": round(step_bytes / (ms_per_step / 1000.0) / 1e9, 1),
           "algorithmic_bytes_per_eval": step_bytes / S,
           "roofline": roofline, "kernels": kernels}

    if not args.no_host_buffers:
        # the same step with the parameters read from and the results written to pageable host memory
        # (the PCIe-inclusive rate; the C ABI's default when no *_ON_DEVICE flag is given)
        progress("one step with host parameters and outputs")
        hflags = N.QQ_ENERGY | N.QQ_GRAD
        xh = np.ascontiguousarray(x)
        eh, gh = np.empty(S), np.empty((S, 2 * p))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for w in range(S // B):
            N.qq_evaluate(pb.handle, p, B, xh[w * B:(w + 1) * B], hflags, ws, ws_bytes, stream, eh[w * B:(w + 1) * B],
                          gh[w * B:(w + 1) * B])
        th = time.perf_counter() - t0
        out["host_buffers"] = {"evals_per_s": round(S / th, 3), "ms_per_step": round(1000.0 * th, 3),
                               "equal_to_device_path": bool(np.array_equal(eh, e_out.cpu().numpy()) and
                                                            np.array_equal(gh, g_out.cpu().numpy())),
                               "note": "one step; parameters copied in and results copied out over PCIe per "
                                       "wave, each call synchronising"}

    # the other legs allocate their own memory: release the timed workspace first
    del ws
    torch.cuda.empty_cache()

    # a plain device copy beside the kernels: the practical bandwidth reference of this GPU
    out["copy_calibration"] = copy_calibration(dev)
    if not args.no_check:
        # sampled parity at full size: complex64 timed path vs the complex128 fused path (both GPU)
        e64 = e_out[:2].cpu().numpy()
        g64 = g_out[:2].cpu().numpy()
        sig = pb.info.sigma_c
        check = {"metric": "energy |dE|/max(|E|, sigma_C); gradient ||dg||_inf/||g||_inf"}
        if args.n == 28 and p == 8:
            # the stored FP64 oracle values of this instance (starts 0 and 1)
            ref = load_golden("regular3_n28_p8_oracle.json")
            er = np.array([st["energy"] for st in ref["starts"]])
            gr = np.array([st["gradient"] for st in ref["starts"]])
            ks = [st["start"] for st in ref["starts"]]
            check["vs_oracle"] = {
                "starts": ks,
                "energy_rel": [float(abs(e64[k] - er[i]) / max(abs(er[i]), sig)) for i, k in enumerate(ks)],
                "grad_rel": [float(np.max(np.abs(g64[k] - gr[i])) / np.max(np.abs(gr[i]))) for i, k in enumerate(ks)]}
        e128, g128 = pb.evaluate(x[:2], grad=True, c128=True)
        check["vs_complex128"] = {"starts": [0, 1],
                                  "energy_rel": float(np.max(np.abs(e64 - e128) / np.maximum(np.abs(e128), sig))),
                                  "grad_rel": float(np.max(np.abs(g64 - g128)) / np.max(np.abs(g128)))}
        out["check"] = check
    if not args.no_plain:
        progress("plain per-gate comparator")
        pb.evaluate_plain(x[0], grad=True)  # warm-up (its allocations and first launches)
        torch.cuda.synchronize()
        times, dev_ms = [], []
        for _ in range(3):
            N.qq_profile_enable(True)
            N.qq_profile_read()
            t0 = time.perf_counter()
            pb.evaluate_plain(x[0], grad=True)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            N.qq_profile_enable(False)
            dev_ms += [r["ms"] for r in N.qq_profile_read() if r["kind"] == 9]
        tp = float(np.median(times))
        out["plain_fp64"] = {"evals_per_s": round(1.0 / tp, 4), "seconds_per_eval": round(tp, 3),
                             "seconds_all": [round(t, 3) for t in times], "speedup": round(value * tp, 2),
                             "device_seconds_per_eval": round(float(np.median(dev_ms)) / 1e3, 3) if dev_ms else None,
                             "speedup_device": round(value * float(np.median(dev_ms)) / 1e3, 2) if dev_ms else None,
                             "timing": "one warm-up, then the median of three calls (each call allocates and "
                                       "frees its own complex128 states); device_seconds_per_eval: HIP events around "
                                       "the call's launch sequence alone, without its allocation",
                             "definition": "complex128, one kernel per gate (phase per layer, RX per qubit and "
                                           "layer, energy reduction, unfused adjoint), one parameter set per call"}
    pb.close()
    torch.cuda.empty_cache()
    if not args.no_aux:
        progress("cost diagonal, probabilities, top-k")
        out["aux"] = aux_kernels(dev, inst, x)
        torch.cuda.empty_cache()
    if not args.no_small:
        progress("12-variable and unit-commitment-shaped workloads")
        out["small_workloads"] = small_workloads(dev)
        torch.cuda.empty_cache()
    if not args.no_uneven:
        progress("uneven batch")
        out["uneven_batch"] = uneven_batch(dev, pinned=pinned_many)
        torch.cuda.empty_cache()
    if not args.no_multi_qpu:
        progress("multi-QPU n = 32")
        out["multi_qpu"] = multi_qpu(dev)
        torch.cuda.empty_cache()
    if not args.no_optimizer:
        progress("depth-progression search")
        out["optimizer"] = optimizer(dev)
        torch.cuda.empty_cache()
    if not args.no_sampling:
        progress("shot sampling")
        out["sampling"] = sampling(dev)
        torch.cuda.empty_cache()
    if not args.no_telegate:
        progress("TeleGate trajectory")
        out["telegate"] = telegate(dev)
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        progress("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline()
        if oracle_cores is not None:
            out["cpu_baseline"]["configs"]["workload4_uneven512"]["multi_core"] = oracle_cores
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
