"""Autotuner for the force step: leaf capacity (ncrit), group size and the
number of persistent walk waves, chosen by timing whole steps on the
caller's workload.

ncrit and the group size change the tree, hence the interaction lists (the
approximation, not the method): every candidate's interactions per particle
and its acceleration difference against the default parameters are reported
beside its time, and `max_rel_diff` rejects candidates that move the forces
more than the caller accepts.  Results are cached in a JSON file keyed by
(architecture, N bucket, number of systems, theta).
"""
from __future__ import annotations

import itertools
import json
import math
import os

from . import mibh

DEFAULT_GRID = {"ncrit": (8, 16, 32), "group_cap": (32, 64), "walk_waves": (2048, 4096)}


def cache_path() -> str:
    return os.environ.get("MIBH_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "mibh", "autotune.json"))


def cache_key(n: int, nsys: int, theta: float) -> str:
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName if torch.cuda.is_available() else "cpu"
    return f"{arch}|n2^{round(math.log2(max(n, 1)))}|nsys{nsys}|theta{theta:g}"


def _time_steps(ctx, pos, mass, offsets, theta, steps, warmup):
    import torch
    for _ in range(warmup):
        ctx.forces_batch(pos, mass, offsets, theta)
    ctx.sync()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(ctx.stream)
    for _ in range(steps):
        acc, pot = ctx.forces_batch(pos, mass, offsets, theta)
    b.record(ctx.stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps, acc


def tune(pos, mass, offsets=None, theta: float = 0.75, grid=None, steps: int = 3, warmup: int = 1,
         max_rel_diff: float | None = None, use_cache: bool = True, write_cache: bool = True):
    """Returns (best parameter dict, list of measured candidates).

    pos/mass are device tensors; offsets (host ints) describe a batch (None: one system)."""
    import torch
    n = int(mass.shape[0])
    offsets = [0, n] if offsets is None else [int(o) for o in offsets]
    nsys = len(offsets) - 1
    key = cache_key(n, nsys, theta)
    path = cache_path()
    if use_cache and os.path.exists(path):
        with open(path) as fh:
            cache = json.load(fh)
        if key in cache:
            return cache[key]["best"], cache[key]["candidates"]
    grid = grid or DEFAULT_GRID
    results = []
    # reference forces: the default parameters (ncrit 16, groups of 64)
    ctx = mibh.Context(n, device=pos.device, max_systems=max(nsys, 1))
    _, ref = _time_steps(ctx, pos, mass, offsets, theta, 1, 0)
    ref = ref.clone()
    del ctx
    for ncrit, gcap, waves in itertools.product(grid["ncrit"], grid["group_cap"], grid["walk_waves"]):
        if ncrit > gcap:
            continue
        ctx = mibh.Context(n, device=pos.device, ncrit=ncrit, group_cap=gcap, walk_waves=waves,
                           max_systems=max(nsys, 1))
        ms, acc = _time_steps(ctx, pos, mass, offsets, theta, steps, warmup)
        st = ctx.stats()
        num = torch.linalg.vector_norm((acc - ref).double(), dim=1)
        den = torch.clamp(torch.linalg.vector_norm(ref.double(), dim=1), min=1e-300)
        diff = float(torch.quantile((num / den)[: 1 << 20], 0.99))
        results.append({"ncrit": ncrit, "group_cap": gcap, "walk_waves": waves, "ms_per_step": ms,
                        "interactions_per_particle": (st["sum_pc"] + st["sum_pp"]) / n,
                        "p99_rel_diff_vs_default": diff})
        del ctx
    ok = [r for r in results if max_rel_diff is None or r["p99_rel_diff_vs_default"] <= max_rel_diff]
    best = min(ok, key=lambda r: r["ms_per_step"])
    best = {k: best[k] for k in ("ncrit", "group_cap", "walk_waves")}
    if write_cache:
        cache = {}
        if os.path.exists(path):
            with open(path) as fh:
                cache = json.load(fh)
        cache[key] = {"best": best, "candidates": results}
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as fh:
            json.dump(cache, fh, indent=1)
    return best, results
