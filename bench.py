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
    (roofline of the dominant kernel: algorithmic bytes / launch time vs 8 TB/s);
  * the plain complex128 per-gate path (one kernel per gate, one parameter
    set per call) on the same GPU, for the speed-up ratio;
  * a sampled parity check of the timed path against the complex128 fused path;
  * the CPU oracle (single thread, FP64) on a bounded sample of the same
    instance family, scaled to n = 28;
  * the uneven batch (512 dense integer QUBOs, n in 10..22, p in 1..6, energy +
    gradient): one autotuned persistent launch (qq_evaluate_many) against one
    qq_evaluate call per problem, both with device-resident inputs and outputs;
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
               for f in ("qq_device.h", "qq_passes.h", "qq_fast.hip", "qq_many.hip", "qq_kernels.hip")]


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


def cpu_baseline(n_sample=22, starts=2, p=8):
    """Oracle energy + adjoint gradient for `starts` starts on an n_sample-node instance of the same family."""
    import numpy as np

    from oracle import oracle as O
    from paper_2606_26297_amd import workloads as W

    inst = W.regular_graph_qubo(n_sample, W.INSTANCE_SEEDS[3])
    d = O.cost_diagonal(inst.H, inst.f, inst.c0)
    x = W.random_params(p, starts, W.PARAM_SEEDS[3])
    t0 = time.perf_counter()
    for b in range(starts):
        O.gradient(d, x[b])
    dt = time.perf_counter() - t0
    scale = (2.0 ** (28 - n_sample)) * 28.0 / n_sample  # work grows as n 2^n
    per_eval_28 = dt / starts * scale
    return {"value": 1.0 / per_eval_28, "unit": "evals/s", "cores": 1, "kind": "oracle",
            "sample": f"{starts} energy+adjoint-gradient evaluations (p={p}) of a {n_sample}-node 3-regular "
                      f"instance of the same generator, single-threaded FP64 C, {dt:.1f} s; scaled to n=28 by "
                      f"2^{28 - n_sample}*28/{n_sample} (work ~ n 2^n)",
            "seconds": dt}


def progress(msg):
    """Stage lines on stderr (stdout carries only the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def uneven_batch(dev, reps=5):
    """The 512-problem uneven batch: persistent launch vs per-problem launches (device-resident)."""
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
    opt, tune_ms = N.qq_autotune_many(handles, ps, bs, flags, None, stream)
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
    del ws
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
    return {"workload": "512 dense integer QUBOs, n ~ U{10..22}, p ~ U{1..6}, 1 parameter set each, energy+grad",
            "persistent_ms": round(1000 * t_many, 3), "persistent_kernel_ms": round(k_ms, 3),
            "persistent_algorithmic_GBps": round(k_bytes / (k_ms / 1000.0) / 1e9, 1),
            "per_problem_ms": round(1000 * t_per, 3), "per_problem_launches": launches,
            "speedup": round(t_per / t_many, 2), "problems_per_s": round(len(items) / t_many, 1),
            "traffic_bytes_per_launch": load_traffic("many_kernel<%s>" % N.DIAG_TYPE_NAMES[pbs[0].info.diag_bytes]),
            "options": opt, "autotune_best_ms": round(tune_ms, 3),
            "energy_rel_vs_per_problem": de}


def aux_kernels(dev, inst, x):
    """Cost diagonal, min/max, probabilities and top-k on the timed instance (one parameter set)."""
    import torch

    from paper_2606_26297_amd import native as N
    from paper_2606_26297_amd.qaoa import Problem

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
    pb = Problem(inst.H, inst.f, inst.c0, device=0)
    caps = [int(c) for c in np.bincount(alloc)]
    cross, remote = pb.set_allocation(alloc, len(caps), caps)
    xt = torch.tensor(x, device=dev)
    out = {"workload": f"dense N(0,1) upper-triangular QUBO, n = {n}, p = {p}, {B} parameter sets, "
                       f"{len(caps)} QPUs x {caps[0]} (contiguous), complex64 energy+grad",
           "cross_terms": cross, "remote_cx_per_layer": remote, "remote_cx_circuit": remote * p}
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
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
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 4 GiB device copy (reference kernel for the traffic counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library runs its hot path on a single MI355X "
              "(sharding over several GPUs is not built). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2606_26297_amd import native as N
    from paper_2606_26297_amd import workloads as W
    from paper_2606_26297_amd.qaoa import Problem

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.uneven_only:
        progress("uneven batch")
        print(json.dumps({"uneven_batch": uneven_batch(dev)}), flush=True)
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
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    N.qq_profile_enable(False)
    recs = N.qq_profile_read()
    wall = t1 - t0
    ms_per_step = 1000.0 * wall / args.steps
    value = S * args.steps / wall

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
    kernels = {k: {"launches": v["launches"], "avg_ms": round(v["ms"] / v["launches"], 4),
                   "GBps": round(v["bytes"] / max(v["ms"], 1e-9) / 1e6, 1)} for k, v in by_kind.items()}

    out = {"metric": METRIC, "value": round(value, 3), "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "c64", "data": "synthetic",
           "config": {"workload": f"regular3_n{args.n}_p{p}_starts{S}", "n": args.n, "p": p, "starts": S,
                      "wave": B, "state": "complex64", "accumulators": "fp64"},
           "schedule": schedule,
           "hbm_GBps_step": round(step_bytes / (ms_per_step / 1000.0) / 1e9, 1),
           "algorithmic_bytes_per_eval": step_bytes / S,
           "roofline": roofline, "kernels": kernels}

    # the other legs allocate their own memory: release the timed workspace first
    del ws
    torch.cuda.empty_cache()

    if args.copy_calibration:
        # a plain copy kernel of known size: its FETCH_SIZE / WRITE_SIZE counters calibrate the
        # counter-derived HBM traffic of the pass kernels
        nbytes = 4 << 30
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = nbytes
        del src, dst
    if not args.no_check:
        # sampled parity at full size: complex64 timed path vs the complex128 fused path (both GPU)
        e64 = e_out[:2].cpu().numpy()
        g64 = g_out[:2].cpu().numpy()
        e128, g128 = pb.evaluate(x[:2], grad=True, c128=True)
        sig = pb.info.sigma_c
        out["check"] = {"vs": "complex128 fused path, starts 0-1",
                        "energy_rel": float(np.max(np.abs(e64 - e128) / np.maximum(np.abs(e128), sig))),
                        "grad_rel": float(np.max(np.abs(g64 - g128)) / np.max(np.abs(g128)))}
    if not args.no_plain:
        progress("plain per-gate comparator")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pb.evaluate_plain(x[0], grad=True)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        out["plain_fp64"] = {"evals_per_s": round(1.0 / tp, 4), "seconds_per_eval": round(tp, 3),
                             "speedup": round(value * tp, 2),
                             "definition": "complex128, one kernel per gate (phase per layer, RX per qubit and "
                                           "layer, energy reduction, unfused adjoint), one parameter set per call"}
    pb.close()
    torch.cuda.empty_cache()
    progress("cost diagonal, probabilities, top-k")
    out["aux"] = aux_kernels(dev, inst, x)
    torch.cuda.empty_cache()
    if not args.no_uneven:
        progress("uneven batch")
        out["uneven_batch"] = uneven_batch(dev)
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
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
