"""Learned warm start for families of barycenter (star) problems.

Pipeline (all arithmetic runs in libgmot; torch only holds device buffers):

1. ``generate``: solve instances cold with the batched solver; collect input
   features (standardised leaf log-marginals) and targets (gauge-fixed leaf
   potentials Lam_(l,0) of the converged state, zero mean per leaf, divided by
   ``out_scale``).
2. ``fit``: train the MLP with the library's forward/backward/Adam kernels on
   mean-squared error.
3. ``compare``: for held-out instances, time cold solves against warm ones
   (features -> network -> potentials -> the same solver), both judged by
   the solver's own stopping rule; instances whose prediction is rejected
   (non-finite) or that fail to converge from the warm start are re-solved
   cold (the fallback).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

from . import Batch, Context, MLP, Problem, star_features, star_targets


@dataclass
class Scaling:
    shift: float
    scale: float
    out_scale: float


@dataclass
class Dataset:
    x: object                 # torch float32 [count, L*n] (device)
    t: object                 # torch float32 [count, L*n] (device)
    scaling: Scaling
    cold_half_sweeps: List[int] = field(default_factory=list)
    cold_seconds: List[float] = field(default_factory=list)


def _torch():
    import torch
    return torch


def solve_cold(ctx: Context, probs: Sequence, batch: int, tol: float, max_steps: int = 200000):
    """Create and solve the given problem descriptions in batches; returns the
    device problems, per-instance results and wall seconds per batch."""
    out_probs, results, walls = [], [], []
    for b0 in range(0, len(probs), batch):
        chunk = [Problem(ctx, p) for p in probs[b0:b0 + batch]]
        bt = Batch(ctx, chunk)
        t0 = time.perf_counter()
        rs = bt.solve(tol=tol, max_steps=max_steps)
        walls.append(time.perf_counter() - t0)
        bt.close()
        out_probs.extend(chunk)
        results.extend(rs)
    return out_probs, results, walls


def generate(ctx: Context, probs: Sequence, batch: int = 512, tol: float = 1e-6, scaling: Optional[Scaling] = None,
             log=None) -> Dataset:
    torch = _torch()
    L = int(probs[0].n_nodes) - 1
    n = int(probs[0].sizes[0])
    count = len(probs)
    x = torch.empty((count, L * n), dtype=torch.float32, device="cuda")
    t = torch.empty((count, L * n), dtype=torch.float32, device="cuda")
    cold_t, cold_s = [], []
    for b0 in range(0, count, batch):
        chunk = [Problem(ctx, p) for p in probs[b0:b0 + batch]]
        bt = Batch(ctx, chunk)
        rs = bt.solve(tol=tol, max_steps=200000)
        bt.close()
        for r in rs:
            if r["status"] != "converged":
                raise RuntimeError(f"training instance did not converge: {r}")
        cold_t.extend(r["t"] for r in rs)
        cold_s.extend(r["seconds"] for r in rs)
        xs, ts = x[b0:b0 + len(chunk)], t[b0:b0 + len(chunk)]
        if scaling is None:
            # standardisation constants from the first chunk's raw values
            star_features(chunk, xs, 0.0, 1.0)
            star_targets(chunk, ts, 1.0)
            torch.cuda.synchronize()
            scaling = Scaling(shift=float(xs.mean().item()), scale=1.0 / max(float(xs.std().item()), 1e-12),
                              out_scale=max(float(ts.std().item()), 1e-12))
        star_features(chunk, xs, scaling.shift, scaling.scale)
        star_targets(chunk, ts, scaling.out_scale)
        for p in chunk:
            p.close()
        if log:
            log(f"generated {min(b0 + batch, count)}/{count}")
    torch.cuda.synchronize()
    return Dataset(x=x, t=t, scaling=scaling, cold_half_sweeps=cold_t, cold_seconds=cold_s)


def fit(ctx: Context, data: Dataset, widths: Sequence[int], epochs: int = 40, batch: int = 256, lr: float = 1e-3,
        seed: int = 0, log=None) -> tuple:
    torch = _torch()
    net = MLP(ctx, widths, seed=seed)
    count = data.x.shape[0]
    usable = count // batch * batch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    losses = []
    for ep in range(epochs):
        perm = torch.randperm(count, device="cuda", generator=g)[:usable]
        lr_ep = lr * 0.5 * (1 + math.cos(math.pi * ep / epochs))
        tot = 0.0
        for b0 in range(0, usable, batch):
            idx = perm[b0:b0 + batch]
            xb = data.x.index_select(0, idx).contiguous()
            tb = data.t.index_select(0, idx).contiguous()
            tot += net.train_step(xb, tb, lr_ep)
        losses.append(tot / max(1, usable // batch))
        if log:
            log(f"epoch {ep}: loss {losses[-1]:.4e}")
    return net, losses


def compare(ctx: Context, net: MLP, scaling: Scaling, probs: Sequence, batch: int = 512, tol: float = 1e-6,
            repeats: int = 1) -> dict:
    """Cold vs warm on the same instances, both as batched solves.  Time of the
    warm path includes building features, the network forward and writing the
    potentials."""
    torch = _torch()
    cold_t, warm_t, cold_wall, warm_wall = [], [], [], []
    rejected = fallback = 0
    for b0 in range(0, len(probs), batch):
        chunk = [Problem(ctx, p) for p in probs[b0:b0 + batch]]
        bt = Batch(ctx, chunk)
        for _ in range(repeats):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc = bt.solve(tol=tol, max_steps=200000, restart=True)
            cold_wall.append(time.perf_counter() - t0)
        cold_t.extend(r["t"] for r in rc)
        for _ in range(repeats):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rej = net.warm_start(chunk, scaling.shift, scaling.scale, scaling.out_scale)
            rw = bt.solve(tol=tol, max_steps=max(r["t"] for r in rc) * 2, restart=False)
            # fallback: anything the warm start could not bring to the tolerance restarts cold
            bad = [i for i, r in enumerate(rw) if r["status"] != "converged"]
            if bad:
                sub = [chunk[i] for i in bad]
                bsub = Batch(ctx, sub)
                rf = bsub.solve(tol=tol, max_steps=200000, restart=True)
                bsub.close()
                for i, r in zip(bad, rf):
                    rw[i] = dict(r, t=r["t"] + rw[i]["t"])
            warm_wall.append(time.perf_counter() - t0)
        rejected += rej
        fallback += len(bad)
        warm_t.extend(r["t"] for r in rw)
        bt.close()
        for p in chunk:
            p.close()
    return {
        "instances": len(probs),
        "cold_half_sweeps_mean": float(np.mean(cold_t)),
        "warm_half_sweeps_mean": float(np.mean(warm_t)),
        "half_sweep_ratio": float(np.mean(cold_t) / np.mean(warm_t)),
        "cold_wall_s": float(np.sum(cold_wall) / repeats),
        "warm_wall_s": float(np.sum(warm_wall) / repeats),
        "time_ratio": float(np.sum(cold_wall) / np.sum(warm_wall)),
        "rejected": int(rejected),
        "fallback": int(fallback),
    }
