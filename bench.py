#!/usr/bin/env python3
"""Benchmark of the bipartite iterative-scaling hot path on one MI355X.

Headline workload (batched-stars-512): 512 independent barycenter stars, each
with a free center and 4-16 constrained leaves (Gaussian-mixture marginals),
n in [128, 2048] points per node on a shared 1D or 2D grid, squared-Euclidean
cost, eps = 1e-2.  One step = every instance solved from the cold start in the
same launches (one captured graph per k half-sweeps, per-instance stop) until
its FP64-judged stopping sum is <= 1e-6, then the FP64 evaluation pass of every
instance in shared launches (dual, primal, transport, both-side stopping
sum).  Inputs are resident in device memory before the timed region.

Metric: edge-iterations/s over the whole batch (an edge-iteration is one edge's
message in one half-sweep), with the device time until the last instance
reaches 1e-6 beside it, and the same instances solved one by one with their
own launches ("plain").  Extras: the 32-node chain (n = 1024, eps = 1e-3), the
256-node random tree (layer-parallel vs per-node launches, explicit-cost
streaming), the learned warm start.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-extras]
       python bench.py --summarize-stats <rocprofv3 kernel_stats.csv>
       python bench.py --summarize-pmc <rocprofv3 counter_collection.csv>
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "edge-iterations/s and time-to-1e-6 marginal error; plain vs batched+warm-start"
# MI355X vector issue: 256 CUs x 4 SIMDs at 2.4 GHz; per SIMD and clock 16 FP64
# lanes (78.6 TFLOP/s FP64 FMA), 32 FP32 lanes (157.3 TFLOP/s) and a quarter of
# that for transcendentals, i.e. SIMD cycles per 64-lane instruction:
SIMD_CLOCKS_PER_S = 256 * 4 * 2.4e9
CYC_FP64, CYC_FP32, CYC_TRANS = 4.0, 2.0, 8.0


def pair_peak_gpairs(dim: int) -> float:
    """ALU peak of the FP32-core message sums (Gpair/s): per pair the least work
    the precision contract allows, dim FP64 FMAs forming the exponent (shift
    folded in), one FP64-to-FP32 conversion, one exp2, one FP32 add."""
    cycles_per_64_pairs = dim * CYC_FP64 + CYC_FP64 + CYC_TRANS + CYC_FP32
    return SIMD_CLOCKS_PER_S * 64 / cycles_per_64_pairs / 1e9


def fma_peak_gpairs() -> float:
    """ALU peak of the uniform-grid message sums (Gpair/s): one FP64 FMA per
    pair (Horner's rule in the row's ratio), 78.6 TFLOP/s / 2."""
    return SIMD_CLOCKS_PER_S * 64 / CYC_FP64 / 1e9


GRID_GROUP_NAME = "k_msg_grid+k_node_sep"


def group_rooflines(st: dict) -> dict:
    """ALU roofline of each kernel group of the node stage that did work, from
    the per-group timing (HIP events around back-to-back repeats of the group
    alone): k_node for D = 1, 2, 3 against the pair peak of its dimension, the
    separable grid kernels (k_sep_pass + k_node_sep) against the one-dimensional
    pair peak (each of their terms is a one-dimensional term), the uniform-grid
    kernels (k_msg_grid + k_node_sep, k_sep_horner + k_node_sep) against one
    FP64 FMA per pair or term, k_node with explicit costs against HBM bandwidth
    at 4 bytes per pair."""
    names = {0: "k_node<explicit>", 1: "k_node<D=1>", 2: "k_node<D=2>", 3: "k_node<D=3>",
             4: "k_sep_pass+k_node_sep", 5: GRID_GROUP_NAME, 6: "k_sep_horner+k_node_sep"}
    n = max(st["msg_launches"], 1)
    out = {}
    for g in range(len(st["group_ms"])):
        ms, pairs = st["group_ms"][g], st["group_pairs"][g]
        if ms <= 0 or pairs <= 0:
            continue
        gps = pairs / (ms / 1e3) / 1e9
        if g == 0:
            ach, peak, unit, bound = 4.0 * gps, HBM_PEAK_GBS, "GB/s", "hbm"
        elif g in (5, 6):
            ach, peak, unit, bound = gps, fma_peak_gpairs(), "Gpair/s", "alu"
        else:
            ach, peak, unit, bound = gps, pair_peak_gpairs(g if g < 4 else 1), "Gpair/s", "alu"
        out[names[g]] = {"bound": bound, "achieved": ach, "peak": peak, "unit": unit, "frac": ach / peak,
                         "ms_per_stage": ms / n, "pairs_per_stage": pairs / n}
    return out


# MI355X HBM3E peak, GB/s
HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")
TRAFFIC_FILE = os.path.join(PROFILES, "k_node_batched512_traffic.txt")
GRID_TRAFFIC_FILE = os.path.join(PROFILES, "k_msg_grid_batched512_traffic.txt")
CHAIN_TRAFFIC_FILE = os.path.join(PROFILES, "k_node_chain32_traffic.txt")
GRID_CHAIN_TRAFFIC_FILE = os.path.join(PROFILES, "k_msg_grid_chain32_traffic.txt")
EXPLICIT_TRAFFIC_FILE = os.path.join(PROFILES, "k_node_explicit_tree256_traffic.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_2406_10849_amd", "csrc", "gmot_kernels.hip")


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def host_info() -> dict:
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "cpu": model}


def kernel_sha() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def measured_traffic(shape, path=None):
    """HBM bytes per node-kernel launch (per node stage for a batch mixing
    support dimensions) from a committed rocprofv3 PMC summary, valid only for
    the kernel source it was taken on and for the node shape (waves per block,
    rows per lane, lane groups) the bench tuned."""
    path = TRAFFIC_FILE if path is None else path
    if not os.path.exists(path):
        return None
    sha, want = None, "shape %d,%d,%d:" % tuple(shape)
    for line in open(path):
        if line.startswith("kernel_sha256_16:"):
            sha = line.split(":", 1)[1].strip()
        elif line.startswith(want) and sha == kernel_sha():
            f = line[len(want):].split()
            try:
                kv = dict(zip(f[0::2], (float(v) for v in f[1::2])))
                return kv["fetch_bytes_per_launch"] + kv["write_bytes_per_launch"]
            except (KeyError, ValueError):
                return None
    return None


# ---------------------------------------------------------------------------
# rocprofv3 output reductions (used to write the summaries under profiles/)
# ---------------------------------------------------------------------------
def summarize_stats(path: str, top: int = 40) -> str:
    """Markdown table of a rocprofv3 --stats kernel summary (CSV)."""
    rows = list(csv.DictReader(open(path)))
    out = ["| kernel | calls | total ns | average ns | % | min ns | max ns |", "|---|---|---|---|---|---|---|"]
    for r in rows[:top]:
        out.append("| `%s` | %s | %s | %.0f | %.2f | %s | %s |" % (
            r["Name"], r["Calls"], r["TotalDurationNs"], float(r["AverageNs"]), float(r["Percentage"]),
            r["MinNs"], r["MaxNs"]))
    return "\n".join(out)


def summarize_pmc(path: str) -> str:
    """Per kernel name: dispatches, the mean counter value per dispatch and the
    largest single dispatch (rocprofv3 --pmc counter_collection CSV, one
    counter per run; with --calib-copy the largest copyBuffer dispatch is the
    1 GiB calibration copy)."""
    acc = {}
    for r in csv.DictReader(open(path)):
        key = (r["Kernel_Name"], r["Counter_Name"])
        a = acc.setdefault(key, [0.0, set(), 0.0])
        v = float(r["Counter_Value"])
        a[0] += v
        a[1].add(r.get("Dispatch_Id", len(a[1])))
        a[2] = max(a[2], v)
    out = ["| kernel | counter | dispatches | mean per dispatch | max dispatch |", "|---|---|---|---|---|"]
    for (k, c), (tot, ids, mx) in sorted(acc.items(), key=lambda kv: -kv[1][0]):
        out.append("| `%s` | %s | %d | %.1f | %.1f |" % (k, c, len(ids), tot / max(len(ids), 1), mx))
    return "\n".join(out)


CALIB_BYTES = 1 << 30   # the --calib-copy device copy: 1 GiB read, 1 GiB written


def pmc_kernel_bytes(path: str, kernel: str, min_frac: float = 0.0):
    """From a rocprofv3 --pmc counter CSV of one byte counter (FETCH_SIZE or
    WRITE_SIZE, KiB per dispatch): (dispatches of the kernel whose name
    starts with `kernel`, their mean in bytes scaled by the calibration copy,
    the scale).  The scale makes the largest copyBuffer dispatch (the 1 GiB
    copy of --calib-copy) read 1 GiB."""
    vals, calib = [], 0.0
    for r in csv.DictReader(open(path)):
        v = float(r["Counter_Value"])
        if r["Kernel_Name"].startswith(kernel):
            vals.append(v)
        elif "copyBuffer" in r["Kernel_Name"]:
            calib = max(calib, v)
    # min_frac > 0 drops launches below that fraction of the largest: ones
    # that did no stage work (every instance had stopped, so the blocks read
    # the loop state and return)
    vals = [v for v in vals if v >= min_frac * max(vals, default=0.0)]
    if not vals or calib <= 0:
        return None
    scale = (CALIB_BYTES / 1024.0) / calib
    return len(vals), statistics.fmean(vals) * 1024.0 * scale, scale


def make_traffic(fetch_csv: str, write_csv: str, kernel: str, shape: str, min_frac: str = "0") -> str:
    """One `shape W,R,H:` line of a traffic file from the two counter runs."""
    f = pmc_kernel_bytes(fetch_csv, kernel, float(min_frac))
    w = pmc_kernel_bytes(write_csv, kernel, float(min_frac))
    if f is None or w is None:
        raise SystemExit(f"no dispatches of {kernel} (or no calibration copy) in the counter files")
    return ("shape %s: fetch_bytes_per_launch %.1f write_bytes_per_launch %.1f dispatches %d\n"
            "calibration %s: FETCH_SIZE scale %.4f, WRITE_SIZE scale %.4f" % (shape, f[1], w[1], f[0], shape, f[2], w[2]))


# ---------------------------------------------------------------------------
# CPU baseline: the FP64 oracle as it stands (message sums in plain C)
# ---------------------------------------------------------------------------
def cpu_baseline(probs, seconds: float, tol: float) -> dict:
    """Sampled instances of the same batch (seeded choice), each solved by the
    oracle from the cold start to the same stopping sum on every host thread,
    until about ``seconds`` of work; then one instance for a fixed number of
    half-sweeps on one thread."""
    from oracle.fast import FastTreeOracle, max_threads
    rng = np.random.default_rng(7)
    order = [int(i) for i in rng.permutation(len(probs))]
    threads = max_threads()
    edges, el, sample = 0, 0.0, []
    for i in order:
        o = FastTreeOracle(probs[i], threads=0)
        t0 = time.perf_counter()
        r = o.solve(tol=tol, max_steps=100000)
        dt = time.perf_counter() - t0
        edges += probs[i].n_edges * r["t"]
        el += dt
        sample.append({"instance": i, "edges": probs[i].n_edges, "n": int(probs[i].sizes[0]), "dim": probs[i].dim,
                       "half_sweeps": r["t"], "status": r["status"], "time_to_tol_s": dt})
        if el >= seconds:
            break
    p1 = probs[order[0]]
    o = FastTreeOracle(p1, threads=1)
    o.tstep()
    steps = 0
    t0 = time.perf_counter()
    while steps < 2 or time.perf_counter() - t0 < min(seconds / 2, 10.0):
        o.tstep()
        steps += 1
    d1 = time.perf_counter() - t0
    return {"value": edges / el, "unit": "edge-iterations/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(sample)} of the 512 stars (seeded choice), each solved from the cold start to a "
                      f"stopping sum <= {tol:g} by the FP64 oracle (message sums in C over {threads} threads), "
                      f"{el:.1f} s in total",
            "instances": sample,
            "one_core": {"value": p1.n_edges * steps / d1, "unit": "edge-iterations/s", "cores": 1,
                         "sample": f"{steps} half-sweeps of instance {order[0]} on one thread, {d1:.1f} s"}}


def cpu_baseline_chain(prob, seconds: float) -> dict:
    """The chain's half-sweeps on the host: every thread, then one thread."""
    from oracle.fast import FastTreeOracle, max_threads
    out = {}
    for th in (0, 1):
        o = FastTreeOracle(prob, threads=th)
        o.tstep()
        steps = 0
        t0 = time.perf_counter()
        while steps < 2 or time.perf_counter() - t0 < seconds:
            o.tstep()
            steps += 1
        dt = time.perf_counter() - t0
        out["all_cores" if th == 0 else "one_core"] = {
            "edge_iterations_per_s": prob.n_edges * steps / dt, "cores": max_threads() if th == 0 else 1,
            "half_sweeps": steps, "s": dt}
    return out


# ---------------------------------------------------------------------------
# headline: the 512 stars in one batch
# ---------------------------------------------------------------------------
def bench_headline(ctx, args, sync) -> tuple:
    from workloads import make_batched_stars
    from paper_2406_10849_amd import Batch, Problem, last_tiles
    probs = make_batched_stars(count=args.batched_count)
    gps = [Problem(ctx, p) for p in probs]
    b = Batch(ctx, gps)
    log("512 stars built; tuning tiles")
    tuned = b.autotune()
    log(f"autotune: {tuned}; tiles: {last_tiles()}")

    def step(timing=False):
        rs = b.solve(tol=args.tol, max_steps=200000, check_every=args.check_every, timing=timing)
        evs = b.evaluate()
        return rs, evs

    for _ in range(max(args.warmup, 0)):
        step()
    sync()
    runs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        runs.append(step())
    sync()
    elapsed = time.perf_counter() - t0
    for k, (rs, evs) in enumerate(runs):
        for i, (r, ev) in enumerate(zip(rs, evs)):
            if r["status"] != "converged" or ev["err_sum"] > args.tol:
                raise RuntimeError(f"step {k} instance {i}: not converged: {r} {ev}")
    edges = [p.n_edges for p in probs]
    edge_iters = sum(sum(e * r["t"] for e, r in zip(edges, rs)) for rs, _ in runs)
    ttt = statistics.median(max(r["seconds"] for r in rs) for rs, _ in runs)
    # the same step with HIP events around every node stage (kernel durations)
    b.stats(reset=True)
    rs_t, _ = step(timing=True)
    st = b.stats()
    groups = group_rooflines(st)
    dom = max(groups, key=lambda g: groups[g]["ms_per_stage"]) if groups else None
    avg_ms = st["msg_ms"] / max(st["msg_launches"], 1)
    shape = (tuned["waves_per_block"], tuned["rows_per_lane"], tuned["lane_groups"])
    traffic = (measured_traffic(shape) if dom == "k_node<D=1>" else
               measured_traffic(shape, GRID_TRAFFIC_FILE) if dom == GRID_GROUP_NAME else None)
    rs0 = runs[-1][0]
    hs = [r["t"] for r in rs0]
    out = {
        "value": edge_iters / elapsed,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "config": {"workload": "batched-stars-512", "instances": len(probs), "edges": int(sum(edges)),
                   "leaves": "4-16 per star", "n": "128-2048 per instance", "dims": "1 or 2 per instance",
                   "eps": probs[0].eps, "tol": args.tol, "cost": "squared-euclidean, on the fly",
                   "marginals": "2-component Gaussian mixtures", "schedule": "bipartite, all instances per launch",
                   "check_every": args.check_every,
                   "pairs_per_half_sweep": int(sum(p.pairs_per_tstep() for p in probs))},
        "time_to_1e-6_s": ttt,
        "half_sweeps_to_1e-6": {"min": int(min(hs)), "median": float(statistics.median(hs)), "max": int(max(hs))},
        "tiles": dict(tuned, **last_tiles()),
        "pairs_per_s": sum(sum(float(p.pairs_per_tstep()) * r["t"] for p, r in zip(probs, rs)) for rs, _ in runs)
                       / elapsed,
        "roofline": dict(groups[dom], kernel=dom, traffic=traffic, stages_timed=st["msg_launches"],
                         node_stage_ms=avg_ms, half_sweep_avg_ms=st["sweep_ms"] / max(st["msg_launches"], 1))
                    if dom else None,
        "kernel_groups": groups,
        "final": {"err_sum_fp64_max": max(ev["err_sum"] for ev in runs[-1][1]),
                  "dual_sum": float(sum(ev["dual"] for ev in runs[-1][1]))},
    }
    if not args.no_extras:
        # plain: each instance on its own (its own plan, graph and launches)
        for g in gps:                                   # plans and graphs built outside the timing
            g.solve(tol=args.tol, max_steps=200000, check_every=args.check_every)
        sync()
        t0 = time.perf_counter()
        rp = [g.solve(tol=args.tol, max_steps=200000, check_every=args.check_every) for g in gps]
        sync()
        t_plain = time.perf_counter() - t0
        assert all(r["status"] == "converged" for r in rp), "per-instance solve did not converge"
        t_batched = elapsed / args.steps
        out["plain"] = {"s": t_plain, "edge_iterations_per_s": sum(e * r["t"] for e, r in zip(edges, rp)) / t_plain,
                        "batched_step_s": t_batched, "speedup_batched_vs_plain": t_plain / t_batched}
    b.close()
    for g in gps:
        g.close()
    return out, probs


# ---------------------------------------------------------------------------
# extras
# ---------------------------------------------------------------------------
def bench_chain(ctx, args, sync) -> dict:
    """The 32-node chain (n = 1024 on a 1D grid, eps = 1e-3, every 4th node
    observed): solves to the FP64-judged stopping sum, the node launch's
    roofline, and the rounding pass of the converged state."""
    from workloads import make_config
    from paper_2406_10849_amd import Problem, last_tiles
    prob = make_config(2)
    g = Problem(ctx, prob)
    tuned = g.autotune()
    for _ in range(2):
        g.solve(tol=args.tol, max_steps=200000, check_every=args.check_every)
    steps = 5
    sync()
    t0 = time.perf_counter()
    rs = []
    for _ in range(steps):
        rs.append(g.solve(tol=args.tol, max_steps=200000, check_every=args.check_every))
        ev = g.evaluate()
    sync()
    el = time.perf_counter() - t0
    assert all(r["status"] == "converged" for r in rs) and ev["err_sum"] <= args.tol
    g.stats(reset=True)
    g.solve(tol=args.tol, max_steps=200000, check_every=args.check_every, timing=True)
    st = g.stats()
    avg_ms = st["msg_ms"] / max(st["msg_launches"], 1)
    ppl = st["msg_pairs"] / max(st["msg_launches"], 1)
    groups = group_rooflines(st)
    dom = max(groups, key=lambda k: groups[k]["ms_per_stage"]) if groups else None
    shape = (tuned["waves_per_block"], tuned["rows_per_lane"], tuned["lane_groups"])
    traffic = (measured_traffic(shape, CHAIN_TRAFFIC_FILE) if dom == "k_node<D=1>" else
               measured_traffic(shape, GRID_CHAIN_TRAFFIC_FILE) if dom == GRID_GROUP_NAME else None)
    # the chain's node stage is one kernel group (one-dimensional uniform grids)
    out = {"workload": "chain-hmm-32node-n1024", "edges": prob.n_edges,
           "edge_iterations_per_s": prob.n_edges * sum(r["t"] for r in rs) / el,
           "time_to_1e-6_s": statistics.median(r["seconds"] for r in rs),
           "half_sweeps_to_1e-6": int(statistics.median(r["t"] for r in rs)), "tiles": dict(tuned, **last_tiles()),
           "dual": ev["dual"], "err_sum_fp64": ev["err_sum"],
           "roofline": dict(groups[dom], kernel=dom, traffic=traffic, node_stage_ms=avg_ms, pairs_per_stage=ppl,
                            stages_timed=st["msg_launches"]) if dom else None}
    rt = []
    for _ in range(5):
        sync()
        t0 = time.perf_counter()
        rr = g.round()
        sync()
        rt.append(time.perf_counter() - t0)
    round_ms = 1e3 * statistics.median(rt)
    pairs = prob.pairs_per_tstep()
    out["rounding"] = {"wall_ms": round_ms, "pair_evaluations": 4 * pairs, "pairs_per_s": 4 * pairs / (round_ms / 1e3),
                       "transport_rounded": rr["transport"], "transport_unrounded": ev["transport"],
                       "err_side": rr["err_side"], "lemma_round_bound": 2 * rr["c_inf"] * rr["err_side"]}
    if not args.no_cpu_baseline:
        out["cpu_oracle"] = cpu_baseline_chain(prob, 5.0)
    g.close()
    return out


def bench_tree(ctx, tol: float, half_sweeps: int, parts=("layer", "per_node", "gauss_seidel", "explicit")) -> dict:
    """The 256-node random tree (n in [256, 4096], 2D grids, eps = 5e-3):
    (a) solved to the stopping sum with every message of a class in one
    launch (layer-parallel), with one launch per node (the same iterates), and
    by node-sequential Gauss-Seidel sweeps (FP64, |V| dependent launches per
    sweep; an edge-iteration there is one of the 2|E| messages of a sweep
    counted per edge, i.e. 2|E| per sweep), and
    (b) with explicit FP32 cost matrices (the squared distances, stored), whose
    message kernel streams 4 bytes per pair from HBM: its roofline is HBM
    bandwidth (the cost set, 4.8 GB per orientation, is far larger than the
    256 MB last-level cache).  `parts` selects among "layer", "per_node" and
    "explicit", "gauss_seidel" (profiling runs take one)."""
    from workloads import make_config, COST_EXPLICIT
    from paper_2406_10849_amd import Problem
    p = make_config(3)
    out = {"workload": "random-tree-256node-2d", "edges": p.n_edges,
           "pairs_per_half_sweep": p.pairs_per_tstep()}
    scheds = [sc for sc in ("layer", "per_node") if sc in parts]
    if scheds:
        g = Problem(ctx, p)
        g.autotune()
        for sched in scheds:
            g.solve(tol=tol, max_steps=200000, schedule=sched)     # graph capture outside the timing
            t0 = time.perf_counter()
            r = g.solve(tol=tol, max_steps=200000, schedule=sched)
            dt = time.perf_counter() - t0
            assert r["status"] == "converged", f"tree ({sched}) did not converge"
            out[sched] = {"s": dt, "half_sweeps": r["t"], "edge_iterations_per_s": p.n_edges * r["t"] / dt}
        if "layer" in scheds:
            # per-group rooflines of the node stage from event-timed half-sweeps
            g.solve(tol=0.0, max_steps=4, timing=True)
            g.stats(reset=True)
            g.solve(tol=0.0, max_steps=half_sweeps, timing=True)
            st = g.stats()
            out["layer"]["kernel_groups"] = group_rooflines(st)
            out["layer"]["half_sweep_avg_ms"] = st["sweep_ms"] / max(st["msg_launches"], 1)
        if len(scheds) == 2:
            out["layer_vs_plain_speedup"] = out["per_node"]["s"] / out["layer"]["s"]
        g.close()
    if "gauss_seidel" in parts:
        g = Problem(ctx, p)
        g.solve(tol=0.0, max_steps=1, schedule="gauss_seidel", check_every=1)   # plan outside the timing
        t0 = time.perf_counter()
        r = g.solve(tol=tol, max_steps=100000, schedule="gauss_seidel", check_every=8)
        dt = time.perf_counter() - t0
        assert r["status"] == "converged", "tree (Gauss-Seidel) did not converge"
        out["gauss_seidel"] = {"s": dt, "sweeps": r["steps"], "precision": "f64", "check_every": 8,
                               "edge_iterations_per_s": 2 * p.n_edges * r["steps"] / dt}
        if "layer" in out:
            out["layer_vs_gauss_seidel_speedup"] = dt / out["layer"]["s"]
        g.close()
    if "explicit" not in parts:
        return out

    cost = []
    for a, b in p.edges:
        X, Y = p.node_support(int(a)), p.node_support(int(b))
        C = np.zeros((X.shape[0], Y.shape[0]))
        for d in range(p.dim):
            C += (X[:, d][:, None] - Y[:, d][None, :]) ** 2
        cost.append(C.astype(np.float32))
    p.cost_kind = COST_EXPLICIT
    p.cost = cost
    g = Problem(ctx, p)
    del cost
    tuned = g.autotune()
    g.solve(tol=0.0, max_steps=4, timing=True)
    g.stats(reset=True)
    g.solve(tol=0.0, max_steps=half_sweeps, timing=True)
    st = g.stats()
    avg_ms = st["msg_ms"] / max(st["msg_launches"], 1)
    pairs = st["msg_pairs"] / max(st["msg_launches"], 1)
    gbs = 4.0 * pairs / (avg_ms / 1e3) / 1e9
    shape = (tuned["waves_per_block"], tuned["rows_per_lane"], tuned["lane_groups"])
    out["explicit_cost"] = {
        "tiles": tuned, "half_sweeps_timed": st["msg_launches"], "pairs_per_launch": pairs,
        "avg_launch_ms": avg_ms, "half_sweep_avg_ms": st["sweep_ms"] / max(st["msg_launches"], 1),
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "traffic": measured_traffic(shape, EXPLICIT_TRAFFIC_FILE),
                     "kernel": "k_node<explicit cost>", "bytes_per_pair": 4}}
    g.close()
    return out


def bench_warm(ctx, tol: float, n_train: int, n_test: int, epochs: int) -> dict:
    """Learned warm start on 8-leaf stars (n = 1024, 1D grid, eps = 1e-2): train
    on solver-generated pairs, then on held-out instances compare (a) each
    instance solved cold on its own (plain), (b) all cold in one batch and (c)
    all warm-started in one batch (features, network and potentials included in
    the time), every solve judged by the iteration's own stopping rule."""
    from workloads import make_warmstart_star
    from paper_2406_10849_amd import Problem, warmstart
    import torch
    t0 = time.perf_counter()
    train = [make_warmstart_star(instance=i) for i in range(n_train)]
    data = warmstart.generate(ctx, train, batch=512, tol=tol)
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    net, losses = warmstart.fit(ctx, data, [8192, 512, 512, 512, 8192], epochs=epochs, batch=256, lr=1e-3)
    torch.cuda.synchronize()
    t_fit = time.perf_counter() - t0
    test = [make_warmstart_star(instance=10 ** 6 + i) for i in range(n_test)]
    res = warmstart.compare(ctx, net, data.scaling, test, batch=n_test, tol=tol)
    # plain: every test instance on its own, cold
    gps = [Problem(ctx, p) for p in test]
    for g in gps:                     # plans and graphs built outside the timing, as for the batch
        g.solve(tol=tol)
    t0 = time.perf_counter()
    rs = [g.solve(tol=tol) for g in gps]
    t_plain = time.perf_counter() - t0
    for g in gps:
        g.close()
    del data
    torch.cuda.empty_cache()
    return dict(res, train_instances=n_train, epochs=epochs, loss_first=losses[0], loss_last=losses[-1],
                generate_s=t_gen, fit_s=t_fit, plain_per_instance_s=t_plain,
                plain_half_sweeps_mean=float(sum(r["t"] for r in rs) / len(rs)),
                speedup_batched_warm_vs_plain=t_plain / res["warm_wall_s"])


def bench_figure(ctx) -> dict:
    """The protocol of the paper's Figure fig:exp for the method itself (the
    globally regularised comparison system is not built): for accuracy
    delta = 0.2, eps = delta / (4 |E| log d) and stopping sum delta' =
    delta / (8 C_inf); half-sweeps until the FP64-judged stopping sum reaches
    delta', then Algorithm round; 5 seeds per point.  Barycenter (log-normal
    leaves on a uniform grid of d points): d varied at |E| = 3, |E| varied at
    d = 10, with Theorem num_iter's bound beside each point.  Wasserstein least
    squares on its modified junction tree (alpha = 10; |E| = J cliques; d = n):
    n varied at J = 3, J varied at n = 10."""
    from workloads import make_lognormal_star, make_wls
    from paper_2406_10849_amd import Problem, JunctionTree
    delta, seeds = 0.2, 5

    def run(make, n_edges, d, c_inf, junction=False):
        eps = delta / (4.0 * n_edges * np.log(d))
        tol = delta / (8.0 * c_inf)
        its, gaps = [], []
        for sd in range(seeds):
            pr = make(eps, sd)
            g = JunctionTree(ctx, pr) if junction else Problem(ctx, pr)
            r = g.solve(tol=tol, max_steps=10 ** 6, precision="fp64")
            assert r["status"] == "converged", r
            its.append(r["t"])
            if not junction:
                gaps.append(g.round()["transport"])
            g.close()
        row = {"d": d, "edges": n_edges, "eps": eps, "delta_prime": tol, "half_sweeps_mean": float(np.mean(its)),
               "half_sweeps": its, "theorem_num_iter_bound": 2 + 88 * n_edges * c_inf / (tol * eps)}
        if gaps:
            row["rounded_transport_mean"] = float(np.mean(gaps))
        return row

    bary_d = [run(lambda e, sd, d=d: make_lognormal_star(3, d, e, instance=sd), 3, d, 1.0)
              for d in (10, 20, 50, 100, 200, 500, 1000)]
    bary_e = [run(lambda e, sd, L=L: make_lognormal_star(L, 10, e, instance=sd), L, 10, 1.0)
              for L in (2, 4, 8, 16, 32, 64)]

    def wls_cinf(J, n):
        return max(float(np.max(c)) for c in make_wls(J=J, n=n, eps=1.0).clique_cost)

    wls_d = [run(lambda e, sd, n=n: make_wls(J=3, n=n, eps=e, instance=sd), 3, n, wls_cinf(3, n), junction=True)
             for n in (5, 10, 20, 40)]
    wls_e = [run(lambda e, sd, J=J: make_wls(J=J, n=10, eps=e, instance=sd), J, 10, wls_cinf(J, 10), junction=True)
             for J in (2, 3, 6, 12)]
    return {"delta": delta, "seeds": seeds, "barycenter_vs_d": bary_d, "barycenter_vs_edges": bary_e,
            "wls_vs_d": wls_d, "wls_vs_edges": wls_e}


def bench_junction(ctx, tol: float) -> dict:
    """Wasserstein least squares (the paper's second experiment, alpha = 10) on
    its modified junction tree: J = 12 observed distributions on n = 32 grid
    points, separators {0, J+1} (1024 joint states) and {j}, eps = 0.05,
    solved to the FP64-judged stopping sum."""
    from workloads import make_wls
    from paper_2406_10849_amd import JunctionTree
    jp = make_wls(J=12, n=32, eps=0.05, instance=0)
    g = JunctionTree(ctx, jp)
    g.solve(tol=tol, max_steps=200000)
    t0 = time.perf_counter()
    r = g.solve(tol=tol, max_steps=200000)
    dt = time.perf_counter() - t0
    ev = g.evaluate()
    pairs = sum(jp.sep_size(a) * jp.sep_size(b) for a, b in jp.cliques)
    return {"workload": "wls-J12-n32 (modified junction tree)", "cliques": jp.n_cliques, "status": r["status"],
            "half_sweeps": r["t"], "s": dt, "time_to_tol_device_s": r["seconds"],
            "clique_iterations_per_s": jp.n_cliques * r["t"] / dt, "pairs_per_half_sweep": pairs,
            "err_sum_fp64": ev["err_sum"], "dual": ev["dual"], "transport": ev["transport"]}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--check-every", type=int, default=16)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one 1 GiB device copy (PMC calibration for HBM byte counters)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the plain comparison, the chain, the tree and the warm start")
    ap.add_argument("--extras", default="chain,tree,warm",
                    help="comma-separated extras to run (chain, tree, tree_layer, tree_explicit, "
                         "tree_gauss_seidel, warm, junction, figure)")
    ap.add_argument("--no-headline", action="store_true",
                    help="skip the headline batch (profiling runs of one extra); prints no bench line")
    ap.add_argument("--batched-count", type=int, default=512)
    ap.add_argument("--tree-half-sweeps", type=int, default=40)
    ap.add_argument("--warm-train", type=int, default=20000)
    ap.add_argument("--warm-test", type=int, default=1024)
    ap.add_argument("--warm-epochs", type=int, default=30)
    ap.add_argument("--summarize-stats", metavar="CSV", help="print a rocprofv3 kernel_stats CSV as markdown")
    ap.add_argument("--summarize-pmc", metavar="CSV", help="print per-dispatch means of a rocprofv3 counter CSV")
    ap.add_argument("--make-traffic", nargs="+", metavar="ARG",
                    help="FETCH_CSV WRITE_CSV KERNEL SHAPE [MIN_FRAC]: print the traffic-file lines of one "
                         "kernel (name prefix) and node shape W,R,H, optionally without launches below "
                         "MIN_FRAC of the largest (ones that did no work)")
    args = ap.parse_args()
    if args.summarize_stats:
        print(summarize_stats(args.summarize_stats))
        return 0
    if args.summarize_pmc:
        print(summarize_pmc(args.summarize_pmc))
        return 0
    if args.make_traffic:
        if len(args.make_traffic) not in (4, 5):
            ap.error("--make-traffic takes FETCH_CSV WRITE_CSV KERNEL SHAPE [MIN_FRAC]")
        print("kernel_sha256_16: %s" % kernel_sha())
        print(make_traffic(*args.make_traffic))
        return 0
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the solver runs on a "
              f"single device; sharding over several GPUs is not built)", file=sys.stderr)
        return 2

    from paper_2406_10849_amd import Context
    try:
        import torch
        sync = torch.cuda.synchronize if torch.cuda.is_available() else (lambda: None)
    except Exception:
        sync = lambda: None  # noqa: E731

    log(f"host: {host_info()}")
    ctx = Context(0)
    extras = [] if args.no_extras else [e.strip() for e in args.extras.split(",") if e.strip()]
    if args.no_headline:
        out, probs = {}, None
    else:
        head, probs = bench_headline(ctx, args, sync)
        out = {"metric": METRIC, "value": head.pop("value"), "unit": "edge-iterations/s", "n_gpus": 1,
               "steps": args.steps, "warmup": args.warmup, "ms_per_step": head.pop("ms_per_step"),
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32exp",
               "data": "synthetic"}
        out.update(head)
        log(f"headline: value {out['value']:.4g} edge-iterations/s, roofline {out['roofline']}")
    if "chain" in extras:
        log("chain: time to 1e-6, node launch roofline, rounding")
        out["chain"] = bench_chain(ctx, args, sync)
        log(f"chain: {out['chain']}")
    tree_parts = set()
    if "tree" in extras:
        tree_parts |= {"layer", "per_node", "gauss_seidel", "explicit"}
    for e in ("tree_layer", "tree_explicit", "tree_gauss_seidel"):
        if e in extras:
            tree_parts.add(e.split("_", 1)[1])
    if tree_parts:
        log("random tree: layer-parallel vs plain schedule, explicit-cost streaming")
        out["tree"] = bench_tree(ctx, args.tol, args.tree_half_sweeps, tree_parts)
        log(f"tree: {out['tree']}")
    if "warm" in extras:
        log("learned warm start")
        out["warm_start"] = bench_warm(ctx, args.tol, args.warm_train, args.warm_test, args.warm_epochs)
        log(f"warm start: {out['warm_start']}")
    if "figure" in extras:
        log("the paper's accuracy-delta protocol (Figure fig:exp), this method's side")
        out["figure"] = bench_figure(ctx)
        log(f"figure: {out['figure']}")
    if "junction" in extras:
        log("Wasserstein least squares on its modified junction tree")
        out["junction"] = bench_junction(ctx, args.tol)
        log(f"junction: {out['junction']}")
    if args.calib_copy:
        import torch
        x = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = 2 * x.numel() * 4
        del x, y
    if args.no_headline:
        return 0
    if not args.no_cpu_baseline and probs is not None:
        log("timing the FP64 oracle on the host")
        out["cpu_baseline"] = cpu_baseline(probs, args.cpu_seconds, args.tol)
        log(f"cpu baseline: {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
