#!/usr/bin/env python3
"""Benchmark of the bipartite iterative-scaling hot path on one MI355X.

Workload: the HMM-like chain (32 nodes, n = 1024 points per node on a 1D grid,
squared-Euclidean cost, eps = 1e-3, every 4th node observed with a 3-component
Gaussian mixture), solved from cold start until the stopping sum of the
Bipartite Iterative Scaling algorithm is <= 1e-6, followed by the FP64
evaluation pass (dual, primal, transport, both-side stopping sum).  One step
= one such solve + evaluation; inputs are resident in device memory before
the timed region.

Metric: edge-iterations/s (an edge-iteration is one edge's message in one
half-sweep; a half-sweep carries |E| = 31 of them), with the device time to
reach 1e-6 reported beside it.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
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
# MI355X HBM3E peak, GB/s
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_node_chain32_traffic.txt")
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


def measured_traffic(shape):
    """HBM bytes per node-kernel launch from the committed rocprofv3 PMC
    summary, valid only for the kernel source it was taken on and for the node
    shape (waves per block, rows per lane, lane groups) the bench tuned."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    sha, want = None, "shape %d,%d,%d:" % shape
    for line in open(TRAFFIC_FILE):
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


def cpu_baseline(prob, seconds: float) -> dict:
    """The FP64 oracle as it stands, on the host, for a bounded number of
    half-sweeps of the same workload."""
    from oracle import TreeOracle
    o = TreeOracle(prob)
    o.tstep()  # first half-sweep also fills the oracle's cost cache
    steps = 0
    t0 = time.perf_counter()
    while True:
        o.tstep()
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    rate = prob.n_edges * steps / el
    return {"value": rate, "unit": "edge-iterations/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} half-sweeps (after one warm-up half-sweep) of the same 32-node chain, "
                      f"FP64 numpy, single thread, {el:.1f} s"}


def bench_batched(ctx, tol: float, count: int) -> dict:
    """Uneven barycenter stars (4-16 leaves, n in [128, 2048], 1D/2D grids,
    eps = 1e-2): all instances advanced by the same launches of one captured
    graph, against each instance solved on its own (its own plan, graph and
    launches), both to the same stopping sum."""
    from workloads import make_batched_stars
    from paper_2406_10849_amd import Batch, Problem
    probs = make_batched_stars(count=count)
    gps = [Problem(ctx, p) for p in probs]
    b = Batch(ctx, gps)
    tuned = b.autotune()
    b.solve(tol=tol, max_steps=200000)              # warm-up (graph capture)
    t0 = time.perf_counter()
    rb = b.solve(tol=tol, max_steps=200000)
    t_batch = time.perf_counter() - t0
    assert all(r["status"] == "converged" for r in rb), "batched solve did not converge"
    for g in gps:                                   # per-instance plans and graphs built outside the timing
        g.solve(tol=tol, max_steps=200000)
    t0 = time.perf_counter()
    rs = [g.solve(tol=tol, max_steps=200000) for g in gps]
    t_single = time.perf_counter() - t0
    assert all(r["status"] == "converged" for r in rs), "per-instance solve did not converge"
    pairs = sum(p.pairs_per_tstep() * r["t"] for p, r in zip(probs, rb))
    edges = sum(p.n_edges * r["t"] for p, r in zip(probs, rb))
    out = {"instances": count, "edges": sum(p.n_edges for p in probs),
           "pairs_per_half_sweep": sum(p.pairs_per_tstep() for p in probs),
           "batched_s": t_batch, "per_instance_s": t_single, "speedup": t_single / t_batch,
           "batched_edge_iterations_per_s": edges / t_batch, "batched_pairs_per_s": pairs / t_batch,
           "max_half_sweeps": max(r["t"] for r in rb), "tiles": tuned}
    b.close()
    for g in gps:
        g.close()
    return out


def bench_tree(ctx, tol: float, half_sweeps: int) -> dict:
    """The 256-node random tree (n in [256, 4096], 2D grids, eps = 5e-3):
    (a) solved to the stopping sum with every message of a class in one
    launch (layer-parallel) and with one launch per message (plain), and
    (b) with explicit FP32 cost matrices (the squared distances, stored), whose
    message kernel streams 4 bytes per pair from HBM: its roofline is HBM
    bandwidth (the cost set, 4.8 GB per orientation, is far larger than the
    256 MB last-level cache)."""
    from workloads import make_config, COST_EXPLICIT
    from paper_2406_10849_amd import Problem
    p = make_config(3)
    out = {"workload": "random-tree-256node-2d", "edges": p.n_edges,
           "pairs_per_half_sweep": p.pairs_per_tstep()}
    g = Problem(ctx, p)
    g.autotune()
    for sched in ("layer", "per_node"):
        g.solve(tol=tol, max_steps=200000, schedule=sched)     # graph capture outside the timing
        t0 = time.perf_counter()
        r = g.solve(tol=tol, max_steps=200000, schedule=sched)
        dt = time.perf_counter() - t0
        assert r["status"] == "converged", f"tree ({sched}) did not converge"
        out[sched] = {"s": dt, "half_sweeps": r["t"], "edge_iterations_per_s": p.n_edges * r["t"] / dt}
    out["layer_vs_plain_speedup"] = out["per_node"]["s"] / out["layer"]["s"]
    g.close()

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
    out["explicit_cost"] = {
        "tiles": tuned, "half_sweeps_timed": st["msg_launches"], "pairs_per_launch": pairs,
        "avg_launch_ms": avg_ms, "half_sweep_avg_ms": st["sweep_ms"] / max(st["msg_launches"], 1),
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "traffic": None, "kernel": "k_node<explicit cost>",
                     "bytes_per_pair": 4}}
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


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--check-every", type=int, default=16)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one 1 GiB device copy (PMC calibration for HBM byte counters)")
    ap.add_argument("--no-extras", action="store_true", help="skip the batched and warm-start comparisons")
    ap.add_argument("--batched-count", type=int, default=512)
    ap.add_argument("--tree-half-sweeps", type=int, default=40)
    ap.add_argument("--warm-train", type=int, default=20000)
    ap.add_argument("--warm-test", type=int, default=1024)
    ap.add_argument("--warm-epochs", type=int, default=30)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the solver runs on a "
              f"single device; sharding over several GPUs is not built)", file=sys.stderr)
        return 2

    from workloads import make_config
    from paper_2406_10849_amd import Context, Problem, last_tiles

    log(f"host: {host_info()}")
    prob = make_config(2)
    n_edges = prob.n_edges
    pairs_per_half_sweep = prob.pairs_per_tstep()
    ctx = Context(0)
    g = Problem(ctx, prob)
    log("workload built; tuning tiles")
    tuned = g.autotune()
    log(f"autotune: {tuned}; tiles: {last_tiles()}")
    for _ in range(max(args.warmup, 0)):
        g.solve(tol=args.tol, max_steps=200000, check_every=args.check_every)
        g.evaluate()
        g.solve(tol=args.tol, max_steps=200000, check_every=args.check_every, timing=True)
    g.stats(reset=True)

    try:
        import torch
        sync = torch.cuda.synchronize if torch.cuda.is_available() else (lambda: None)
    except Exception:
        sync = lambda: None  # noqa: E731

    def timed_region(timing: bool):
        sync()
        runs = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            r = g.solve(tol=args.tol, max_steps=200000, check_every=args.check_every, timing=timing)
            ev = g.evaluate()
            runs.append((r, ev))
        sync()
        return runs, time.perf_counter() - t0

    # region 1: the product configuration (graph replay) -> value
    runs, elapsed = timed_region(False)
    # region 2: the same steps with HIP events around every stage -> kernel durations
    g.stats(reset=True)
    runs_t, elapsed_t = timed_region(True)
    st = g.stats()
    for i, (r, ev) in enumerate(runs + runs_t):
        if r["status"] != "converged" or ev["err_sum"] > args.tol:
            log(f"step {i}: not converged: {r} {ev}")
            return 1
    half_sweeps = [r["t"] for r, _ in runs]      # half-sweeps computed, including the one that passed the test
    edge_iters = n_edges * sum(half_sweeps)
    value = edge_iters / elapsed
    ttt = statistics.median(r["seconds"] for r, _ in runs)
    last_r, last_ev = runs[-1]
    log(f"solve: {last_r}")
    log(f"eval: {last_ev}")
    log(f"stats: {st}")

    D = prob.dim
    peak = pair_peak_gpairs(D)
    avg_ms = st["msg_ms"] / max(st["msg_launches"], 1)
    pairs_per_launch = st["msg_pairs"] / max(st["msg_launches"], 1)
    achieved = pairs_per_launch / (avg_ms / 1e3) / 1e9 if avg_ms > 0 else 0.0
    traffic = measured_traffic((tuned["waves_per_block"], tuned["rows_per_lane"], tuned["lane_groups"]))
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "edge-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32exp",
        "data": "synthetic",
        "config": {"workload": "chain-hmm-32node-n1024", "nodes": prob.n_nodes, "edges": n_edges,
                   "n": int(prob.sizes[0]), "dim": D, "eps": prob.eps, "tol": args.tol,
                   "cost": "squared-euclidean, on the fly", "observed": "every 4th node, 3-comp GM",
                   "schedule": "bipartite (layer-parallel)", "check_every": args.check_every},
        "time_to_1e-6_s": ttt,
        "half_sweeps_to_1e-6": int(statistics.median(half_sweeps)),
        "value_event_timed_region": n_edges * sum(r["t"] for r, _ in runs_t) / elapsed_t,
        "tiles": dict(tuned, **last_tiles()),
        "pairs_per_s": pairs_per_half_sweep * sum(half_sweeps) / elapsed,
        "final": {"err_sum_fp64": last_ev["err_sum"], "err_max_fp64": last_ev["err_max"],
                  "dual": last_ev["dual"], "primal": last_ev["primal"], "transport": last_ev["transport"]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Gpair/s",
                     "frac": achieved / peak, "traffic": traffic,
                     "kernel": "k_node", "avg_launch_ms": avg_ms, "pairs_per_launch": pairs_per_launch,
                     "launches_timed": st["msg_launches"],
                     "half_sweep_avg_ms": st["sweep_ms"] / max(st["msg_launches"], 1)},
    }
    # rounding of the converged state onto the constraint set (Algorithm round):
    # four FP64 row passes over recomputed plan entries (row sums of both
    # orientations, column scaling, final pass), outside the timed region
    rt = []
    for _ in range(5):
        sync()
        t0 = time.perf_counter()
        rr = g.round()
        sync()
        rt.append(time.perf_counter() - t0)
    round_ms = 1e3 * statistics.median(rt)
    out["rounding"] = {"wall_ms": round_ms, "pair_evaluations": 4 * pairs_per_half_sweep,
                       "pairs_per_s": 4 * pairs_per_half_sweep / (round_ms / 1e3),
                       "transport_rounded": rr["transport"], "transport_unrounded": last_ev["transport"],
                       "err_side": rr["err_side"], "lemma_round_bound": 2 * rr["c_inf"] * rr["err_side"]}
    log(f"rounding: {out['rounding']}")
    if not args.no_extras:
        log("batched stars: one graph for all instances vs per-instance launches")
        out["batched"] = bench_batched(ctx, args.tol, args.batched_count)
        log(f"batched: {out['batched']}")
        log("random tree: layer-parallel vs plain schedule, explicit-cost streaming")
        out["tree"] = bench_tree(ctx, args.tol, args.tree_half_sweeps)
        log(f"tree: {out['tree']}")
        log("learned warm start")
        out["warm_start"] = bench_warm(ctx, args.tol, args.warm_train, args.warm_test, args.warm_epochs)
        log(f"warm start: {out['warm_start']}")
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host")
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_seconds)
    if args.calib_copy:
        import torch
        x = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = 2 * x.numel() * 4
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
