"""Benchmark of one full Barnes-Hut force step on one MI355X.

Default workload: Plummer sphere of N = 2^22 equal-mass particles (seed 3,
Henon units), theta = 0.75, ncrit 16, groups of <= 64, float32 interactions,
float64 multipoles.  A step is the whole hot path on inputs already resident
in HBM: bounding cube, keys, radix sort, reorder, octree + groups, multipoles,
MAC preparation and the group walk, with results in the caller's order.

Prints ONE JSON line on stdout: particles/s of the full step (whole job),
interactions/s, per-stage times (HIP events on the library's stream), the
walk kernel's roofline (float32 vector ALU bound) and the float64 CPU
oracle's throughput on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

F_PC = 53  # flops per particle-cell interaction (monopole + traceless quadrupole, rsqrt = 1)
F_PP = 20  # flops per particle-particle interaction (rsqrt = 1)
PEAK_FP32_TFLOPS = 157.3  # MI355X published float32 vector peak (256 CU x 2.4 GHz x 256 flop/clk)
WALK_SOURCES = ("paper_1204_2280_amd/csrc/walk_kernel.hip", "paper_1204_2280_amd/csrc/mibh_device.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "walk_hbm_traffic.json")


PEAK_HBM_GBS = 8000.0  # MI355X published HBM3E bandwidth

# Algorithmic HBM bytes of the tree stages: per particle, per radix pass and per cell.
#   sorting: bounding box reads x, y, z, m (16); keys read them again and write the
#     key (8) and the packed record (16); each of the 8 radix passes (60-bit keys in
#     8-bit digits) reads the key for the histogram (8), reads key + index (12) and
#     writes them (12);
#   moving: index (4), gathered record (16), written record (16);
#   tree construction: keys and the common-prefix byte read (9), level record
#     written and read (8), groups written (8), plus one 16-byte topology record per cell;
#   multipoles: sorted records read (16) plus per cell the topology (16), float64
#     moments, delta and l' written (96) and read back by the parent (96), the
#     particle box (24) and the walk data (48) written.
HBM_B_PER_PARTICLE = {"sorting": 16 + 40 + 8 * 32, "moving": 36, "tree_construction": 25, "multipoles": 16}
HBM_B_PER_CELL = {"tree_construction": 16, "multipoles": 16 + 96 + 96 + 24 + 48}


def hbm_stages(stage_ms, n, ncells):
    """Achieved algorithmic bandwidth of each tree stage against 8 TB/s."""
    out = {}
    for k, bp in HBM_B_PER_PARTICLE.items():
        ms = stage_ms[k] + (stage_ms["mac_prep"] if k == "multipoles" else 0.0)
        b = bp * n + HBM_B_PER_CELL.get(k, 0) * ncells
        gbs = b / (ms * 1e-3) / 1e9
        out[k] = {"bytes": b, "ms": ms, "GB/s": gbs, "frac": gbs / PEAK_HBM_GBS}
    return out


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def walk_source_hash() -> str:
    """Hash of the walk kernel's code: its sources with comments and blank
    lines removed, so that a comment edit keeps the recorded counters."""
    import re
    h = hashlib.sha256()
    for f in WALK_SOURCES:
        with open(os.path.join(ROOT, f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        lines = [ln.rstrip() for ln in text.splitlines()]
        h.update("\n".join(ln for ln in lines if ln).encode())
    return h.hexdigest()


def measured_traffic(workload: str):
    """HBM bytes per walk launch from committed rocprofv3 counter runs, if they
    were taken on the current walk kernel source and this workload."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != walk_source_hash() or t.get("workload") != workload:
        return None
    return t.get("bytes_per_launch")


def fma_ceiling(dev, blocks=256 * 4 * 8, iters=20000):
    """Rate (TFLOP/s) that plain float32 fused multiply-adds reach on this GPU:
    the library's probe kernel, 8 waves per SIMD, 32 independent accumulators
    per lane; the best of three launches timed with HIP events."""
    import torch
    from paper_1204_2280_amd import mibh
    out = torch.empty(blocks * 2048, dtype=torch.float32, device=dev)
    s = torch.cuda.current_stream(dev)
    mibh.fma_probe(out, blocks, iters // 10)
    best = float("inf")
    for _ in range(3):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        mibh.fma_probe(out, blocks, iters)
        e1.record(s)
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return blocks * 64 * iters * 64 / (best * 1e-3) / 1e12


def cpu_baseline(pos, mass, theta, n_ranges=16, frac=1 / 2):
    """The float64 oracle on the host cores: full tree build on all particles
    plus the walk of a sample of groups, the walk time scaled to all groups."""
    import numpy as np
    import oracle
    t0 = time.perf_counter()
    T = oracle.Tree(pos, mass)
    t_build = time.perf_counter() - t0
    ng = T.ngroups
    width = max(1, int(ng * frac / n_ranges))
    starts = np.linspace(0, ng - width, n_ranges).astype(np.int64)
    t_walk = 0.0
    sampled = 0
    for s in starts:
        t0 = time.perf_counter()
        T.walk(theta, groups=(int(s), int(s) + width))
        t_walk += time.perf_counter() - t0
        sampled += width
    t_step = t_build + t_walk * ng / sampled
    # the paper's host had 4 cores: the same estimate with 4 threads on an eighth of the groups
    width4 = max(1, width // 4)
    t_walk4 = 0.0
    for s in starts:
        t0 = time.perf_counter()
        T.walk(theta, groups=(int(s), int(s) + width4), nthreads=4)
        t_walk4 += time.perf_counter() - t0
    t_step4 = t_build + t_walk4 * ng / (width4 * n_ranges)
    n = len(mass)
    # complete oracle steps at the smaller sizes (no sampling): 3 runs at 2^15, 1 at 2^20
    from paper_1204_2280_amd import workloads
    full = {}
    for nn, seed, runs in ((1 << 15, 1, 3), (1 << 20, 2, 1)):
        ps, _, ms = workloads.plummer(nn, seed, with_velocities=False)
        best = None
        for _ in range(runs):
            t0 = time.perf_counter()
            Ts = oracle.Tree(ps, ms)
            t1 = time.perf_counter()
            Ts.walk(theta)
            t2 = time.perf_counter()
            if best is None or t2 - t0 < best[0] + best[1]:
                best = (t1 - t0, t2 - t1)
        full[f"plummer_n{nn}_seed{seed}"] = {"build_s": best[0], "walk_s": best[1],
                                             "particles_per_s": nn / (best[0] + best[1]), "runs": runs}
    return {
        "value": n / t_step,
        "value_4_threads": n / t_step4,
        "unit": "particles/s",
        "cores": oracle.num_threads(),
        "cpu_model": cpu_model(),
        "kind": "oracle",
        "complete_steps": full,
        "sample": (f"float64 oracle: full tree build of all {n} particles ({t_build:.2f} s, one thread) + "
                   f"walk of {sampled} of {ng} groups in {n_ranges} ranges ({t_walk:.2f} s), walk time "
                   f"scaled by {ng / sampled:.1f}; estimated step {t_step:.1f} s; with 4 threads "
                   f"{width4 * n_ranges} groups in {t_walk4:.2f} s, estimated step {t_step4:.1f} s"),
    }


def bench_variant_kahan(pos, mass, theta, steps, warmup, rounds=3):
    """Same workload with compensated accumulation: Kahan across the list
    evaluations (MIBH_KAHAN) and per term (MIBH_KAHAN_TERM), timed in
    alternation with the plain walk (medians of `rounds` rounds)."""
    import numpy as np
    import torch
    from paper_1204_2280_amd import mibh
    n = len(mass)
    dev = torch.device("cuda", 0)
    p = torch.from_numpy(pos).to(dev)
    m = torch.from_numpy(mass).to(dev)
    ctxs = {name: mibh.Context(n, device=dev, precision=prec)
            for name, prec in (("plain", mibh.PLAIN), ("kahan", mibh.KAHAN), ("kahan_term", mibh.KAHAN_TERM))}
    times = {name: [] for name in ctxs}
    for name, ctx in ctxs.items():
        for _ in range(warmup):
            ctx.forces(p, m, theta)
        ctx.sync()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(rounds):
        for name, ctx in ctxs.items():
            a.record(ctx.stream)
            for _ in range(steps):
                ctx.forces(p, m, theta)
            b.record(ctx.stream)
            torch.cuda.synchronize()
            times[name].append(a.elapsed_time(b) / steps)
    del ctxs
    out = {}
    for name, t in times.items():
        ms = float(np.median(t))
        out[name] = {"ms_per_step": ms, "particles_per_s": n / (ms * 1e-3)}
    for name in ("kahan", "kahan_term"):
        out[name]["cost_vs_plain"] = out[name]["ms_per_step"] / out["plain"]["ms_per_step"] - 1.0
    out["timing"] = f"{rounds} alternating rounds x {steps} steps per mode, medians"
    return out


def bench_variant_ensemble(theta, steps, warmup, w16, nsys=64, seed=4, rounds=3):
    """Batched ensemble (uneven N, half Plummer, half Hernquist truncated at 50):
    one graph-replayed batched step vs one single-system step per system; the
    graph-replayed step in four configurations (plain or Kahan accumulation,
    Morton or learned-estimator queue order) timed in alternation, medians of
    `rounds` rounds.  Returns (record, outputs): outputs holds the plain and
    the Kahan + estimator forces for the oracle comparison of the CPU leg."""
    import numpy as np
    import torch
    from paper_1204_2280_amd import mibh, workloads
    pos, mass, off = workloads.ensemble(nsys, seed)
    n = int(off[-1])
    dev = torch.device("cuda", 0)
    stream = torch.cuda.Stream(device=dev)
    p = torch.from_numpy(pos).to(dev)
    m = torch.from_numpy(mass).to(dev)
    acc = torch.empty((n, 3), dtype=torch.float32, device=dev)
    pot = torch.empty((n,), dtype=torch.float32, device=dev)
    ctx = mibh.Context(n, device=dev, stream=stream, max_systems=nsys)
    with torch.cuda.stream(stream):
        ctx.graph_capture(p, m, off, theta, acc, pot)
        for _ in range(warmup):
            ctx.graph_launch()
        ctx.sync()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(steps):
            ctx.graph_launch()
        b.record(stream)
        torch.cuda.synchronize()
        ms_batch = a.elapsed_time(b) / steps
        ctx.sync()
        st = ctx.stats()
        # the same systems one at a time (eager, one context sized for the largest)
        single = mibh.Context(int(np.max(np.diff(off))), device=dev, stream=stream)
        views = [(p[off[k]:off[k + 1]], m[off[k]:off[k + 1]], acc[off[k]:off[k + 1]], pot[off[k]:off[k + 1]])
                 for k in range(nsys)]
        for _ in range(warmup):
            for (pk, mk, ak, qk) in views:
                single.forces(pk, mk, theta, ak, qk)
        single.sync()
        a.record(stream)
        for _ in range(steps):
            for (pk, mk, ak, qk) in views:
                single.forces(pk, mk, theta, ak, qk)
        b.record(stream)
        torch.cuda.synchronize()
        ms_seq = a.elapsed_time(b) / steps
        # autotuned parameters (ncrit, group size, walk waves), graph-replayed
        from paper_1204_2280_amd import autotune
        best, cands = autotune.tune(p, m, off, theta, steps=2, warmup=1, max_rel_diff=2e-3, use_cache=False,
                                    write_cache=False)
        tuned = mibh.Context(n, device=dev, stream=stream, max_systems=nsys, **best)
        tuned.graph_capture(p, m, off, theta, acc, pot)
        tuned.graph_launch()
        tuned.sync()
        a.record(stream)
        for _ in range(steps):
            tuned.graph_launch()
        b.record(stream)
        torch.cuda.synchronize()
        ms_tuned = a.elapsed_time(b) / steps
        del tuned, single
        # the four configurations, one context each, timed in alternation
        cfgs = {}
        for name, prec, w in (("plain_morton", mibh.PLAIN, None), ("kahan_morton", mibh.KAHAN, None),
                              ("plain_estimator", mibh.PLAIN, w16), ("kahan_estimator", mibh.KAHAN, w16)):
            c = mibh.Context(n, device=dev, stream=stream, max_systems=nsys, precision=prec)
            if w is not None:
                c.set_queue_order(mibh.ORDER_ESTIMATOR, w)
            ca = torch.empty((n, 3), dtype=torch.float32, device=dev)
            cq = torch.empty((n,), dtype=torch.float32, device=dev)
            c.graph_capture(p, m, off, theta, ca, cq)
            for _ in range(warmup):
                c.graph_launch()
            cfgs[name] = (c, ca, cq, [])
        for _ in range(rounds):
            for name, (c, ca, cq, times) in cfgs.items():
                c.graph_launch()
                a.record(stream)
                for _ in range(steps):
                    c.graph_launch()
                b.record(stream)
                torch.cuda.synchronize()
                times.append(a.elapsed_time(b) / steps)
        configs = {name: {"ms_per_step": float(np.median(t)), "particles_per_s": n / (float(np.median(t)) * 1e-3)}
                   for name, (_, _, _, t) in cfgs.items()}
        outputs = {name: (cfgs[name][1].cpu().numpy(), cfgs[name][2].cpu().numpy())
                   for name in ("plain_morton", "kahan_estimator")}
        del cfgs
    rec = {"workload": f"ensemble_{nsys}sys_seed{seed}_n{n}_theta{theta:g}", "n": n, "nsys": nsys,
            "autotuned": best, "ms_per_step_tuned_graph": ms_tuned,
            "particles_per_s_tuned_graph": n / (ms_tuned * 1e-3),
            "ms_per_step_batched_graph": ms_batch, "particles_per_s_batched_graph": n / (ms_batch * 1e-3),
            "ms_per_step_sequential": ms_seq, "particles_per_s_sequential": n / (ms_seq * 1e-3),
            "speedup": ms_seq / ms_batch, "interactions_per_s_batched":
                (st["sum_pc"] + st["sum_pp"]) / (ms_batch * 1e-3),
            "graph_configs": configs,
            "graph_configs_timing": f"{rounds} alternating rounds x {steps} replays per configuration, medians"}
    return rec, outputs


def _p99_rel(a, ref):
    """99th percentile (nearest rank) of |a_i - ref_i| / |ref_i| over rows."""
    import numpy as np
    a = np.asarray(a, np.float64)
    ref = np.asarray(ref, np.float64)
    num = np.linalg.norm(a - ref, axis=1) if a.ndim == 2 else np.abs(a - ref)
    den = np.linalg.norm(ref, axis=1) if ref.ndim == 2 else np.abs(ref)
    e = np.sort(num / np.where(den > 0, den, 1.0))
    return float(e[int(np.ceil(0.99 * e.size)) - 1])


def cpu_baseline_ensemble(theta, outputs, nsys=64, seed=4):
    """The float64 oracle on the ensemble: every system's tree and walk, timed
    on the host cores; the GPU's plain and Kahan + estimator forces are scored
    against its results (relative error, 99th percentile over all particles)."""
    import numpy as np
    import oracle
    from paper_1204_2280_amd import workloads
    pos, mass, off = workloads.ensemble(nsys, seed)
    n = int(off[-1])
    acc = np.empty((n, 3))
    pot = np.empty(n)
    t0 = time.perf_counter()
    for k in range(nsys):
        a, b = int(off[k]), int(off[k + 1])
        T = oracle.Tree(pos[a:b], mass[a:b])
        T.walk(theta)
        acc[a:b], pot[a:b] = T.forces()
        del T
    t = time.perf_counter() - t0
    return {"value": n / t, "unit": "particles/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"the whole ensemble: {nsys} systems, {n} particles, tree and walk in {t:.2f} s",
            "acc_p99_vs_oracle": {k: _p99_rel(v[0], acc) for k, v in outputs.items()},
            "pot_p99_vs_oracle": {k: _p99_rel(v[1], pot) for k, v in outputs.items()}}


def train_estimator(pos_train, mass_train, theta):
    """The learned work estimator, trained on the GPU on the per-group counts of
    Plummer spheres of 2^15 (seed 1), 2^20 (seed 2) and the headline 2^22 system
    (given): returns its float16 weights."""
    import torch
    from paper_1204_2280_amd import estimator, mibh, workloads
    dev = torch.device("cuda", 0)
    xs, ts = [], []
    for pt, mt in [workloads.plummer(1 << 15, 1, with_velocities=False)[::2],
                   workloads.plummer(1 << 20, 2, with_velocities=False)[::2], (pos_train, mass_train)]:
        nt = len(mt)
        c = mibh.Context(nt, device=dev)
        c.forces(torch.from_numpy(pt).to(dev), torch.from_numpy(mt).to(dev), theta)
        c.sync()
        x, t = estimator.collect(c, theta)
        xs.append(x)
        ts.append(t)
        del c
    _, w16, _ = estimator.train(torch.cat(xs), torch.cat(ts), steps=1000, batch=1024, lr=3e-3)
    return w16


def bench_variant_queue_order(w16, theta, steps, rounds=5):
    """Queue orders on two Plummer spheres of 2^21 particles each (seeds 5 and 6,
    10 apart): Morton; longest-processing-time first by the exact counts of the
    previous walk of the same tree; and by the learned estimator.  The three are
    timed in alternation (rounds x steps each) from the library's stage events;
    "order_and_walk_ms" is the MAC-data stage (which holds the estimator's
    feature and forward kernels and the ordering kernels) plus the walk, the
    part of a step that the order changes; the estimator and Morton steps are
    also timed whole.  Medians over all timed steps."""
    import numpy as np
    import torch
    from paper_1204_2280_amd import estimator, mibh, workloads
    dev = torch.device("cuda", 0)
    pos, mass = workloads.two_plummers(1 << 21)
    n = len(mass)
    p = torch.from_numpy(pos).to(dev)
    m = torch.from_numpy(mass).to(dev)
    ctx = mibh.Context(n, device=dev)

    def run_mode(mode):
        if mode == "morton":
            ctx.set_queue_order(mibh.ORDER_MORTON)
            return lambda: ctx.forces(p, m, theta)
        if mode == "estimator":
            ctx.set_queue_order(mibh.ORDER_ESTIMATOR, w16)
            return lambda: ctx.forces(p, m, theta)
        ctx.set_queue_order(mibh.ORDER_EXACT)
        ctx.forces(p, m, theta)
        ctx.compute_forces(theta)  # exact counts of this tree
        return lambda: ctx.compute_forces(theta)

    rec = {k: [] for k in ("morton", "estimator", "exact")}
    for r in range(rounds + 1):
        for mode in rec:
            fn = run_mode(mode)
            fn()
            ctx.sync()
            ctx.profile_begin(steps)
            for _ in range(steps):
                fn()
            got = ctx.profile_read()
            if r > 0:  # the first alternation warms every mode up
                rec[mode].extend(got)
    out = {}
    for mode, rows in rec.items():
        med = {k: float(np.median([x[k] for x in rows])) for k in rows[0]}
        d = {"walk_ms": med["walk"], "mac_prep_ms": med["mac_prep"],
             "order_and_walk_ms": float(np.median([x["mac_prep"] + x["walk"] for x in rows]))}
        if mode != "exact":
            d["step_ms"] = float(np.median([sum(x.values()) for x in rows]))
        out[mode] = d
    out["exact"]["note"] = "repeated walks of one tree (the counts of a new tree are not known before its walk)"
    x, t = estimator.collect(ctx, theta)
    out["estimator"]["quality"] = estimator.evaluate(w16, x, t)
    out["estimator_gain_ms"] = {
        "vs_morton": out["morton"]["order_and_walk_ms"] - out["estimator"]["order_and_walk_ms"],
        "vs_exact": out["exact"]["order_and_walk_ms"] - out["estimator"]["order_and_walk_ms"]}
    del ctx
    out["workload"] = f"two_plummers_2x2^21_seeds5_6_sep10_theta{theta:g}"
    out["timing"] = f"{rounds} alternating rounds x {steps} steps per order, medians"
    return out


def bench_variant_leapfrog(n, seed, theta, steps):
    """Shared-time-step kick-drift-kick driver on the same Plummer sphere with
    its velocities: milliseconds per step (one force step and two fused
    kick/drift launches; the initial force evaluation is timed too and spread
    over the steps) and the float64 energy drift over the run (dt = 1/128,
    softening eps = 0.01: with no softening the closest pairs of 2^22 bodies
    need far smaller steps than a shared dt gives them)."""
    import torch
    from paper_1204_2280_amd import mibh, workloads
    pos, vel, mass = workloads.plummer(n, seed)
    dev = torch.device("cuda", 0)
    P, V, M = (torch.from_numpy(t.copy()).to(dev) for t in (pos, vel, mass))
    eps2 = 1e-4
    ctx = mibh.Context(n, device=dev, eps2=eps2)
    dt = 1.0 / 128
    ctx.leapfrog(P, V, M, theta, dt, 1)  # warm-up
    P.copy_(torch.from_numpy(pos))
    V.copy_(torch.from_numpy(vel))
    ctx.sync()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(ctx.stream)
    ctx.leapfrog(P, V, M, theta, dt, steps)
    b.record(ctx.stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    P.copy_(torch.from_numpy(pos))
    V.copy_(torch.from_numpy(vel))
    _, _, log = ctx.leapfrog(P, V, M, theta, dt, steps, log_every=max(1, steps // 4))
    E = log[:, 1] + log[:, 2]
    del ctx
    return {"workload": f"plummer_n{n}_seed{seed}_theta{theta:g}_dt{dt:g}_eps2{eps2:g}", "steps": steps,
            "ms_per_step": ms, "particles_per_s": n / (ms * 1e-3),
            "energy_log": [[float(t), float(T), float(W)] for t, T, W in log],
            "rel_energy_drift": float(abs(E[-1] - E[0]) / abs(E[0]))}


def bench_variant_block_steps(n, seed, theta, shared_ms):
    """Block time steps on the same Plummer sphere with velocities (softening
    eps = 0.01): steps of dt_max = 1/16 in 16 ticks (levels 0..4, criterion
    dt = 0.1 sqrt(0.1 / |a|)), refits between work-triggered rebuilds
    (tolerance 0.25).  A run starts with a force evaluation of every particle;
    the steady time per dt_max is (t(3 steps) - t(1 step)) / 2.  It is
    compared with 16 shared steps of the smallest step dt_max/16 (every
    particle updated every tick) at the leapfrog driver's time per step."""
    import torch
    from paper_1204_2280_amd import mibh, workloads
    pos, vel, mass = workloads.plummer(n, seed)
    dev = torch.device("cuda", 0)
    P, V, M = (torch.from_numpy(t.copy()).to(dev) for t in (pos, vel, mass))
    ctx = mibh.Context(n, device=dev, eps2=1e-4)
    args = (theta, 1.0 / 16, 4, 0.1, 0.1)

    def run(nbig):
        P.copy_(torch.from_numpy(pos))
        V.copy_(torch.from_numpy(vel))
        ctx.sync()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(ctx.stream)
        _, _, lev, st, _ = ctx.block_run(P, V, M, *args, nbig, log=False)
        b.record(ctx.stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b), lev, st

    run(1)  # warm-up
    t1, _, st1 = run(1)
    t3, lev, st3 = run(3)
    steady = (t3 - t1) / 2
    hist = torch.bincount(lev.to(torch.int64), minlength=5).cpu().tolist()
    ticks = block_tick_walks(ctx, P, V, M, lev, theta, args[1] / 16)
    # the same steps rebuilding the tree before every walk (no refits)
    args_rb = args
    def run_rb(nbig):
        P.copy_(torch.from_numpy(pos))
        V.copy_(torch.from_numpy(vel))
        ctx.sync()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(ctx.stream)
        _, _, _, st, _ = ctx.block_run(P, V, M, *args_rb, nbig, rebuild_tol=-1.0, log=False)
        b.record(ctx.stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b), st
    run_rb(1)
    r1, _ = run_rb(1)
    r3, rst3 = run_rb(3)
    steady_rb = (r3 - r1) / 2
    del ctx
    upd = (st3["active_updates"] - st1["active_updates"]) / 2
    out = {"workload": f"plummer_n{n}_seed{seed}_theta{theta:g}_eps2{1e-4:g}_dtmax{1 / 16:g}_levels0-4",
           "schedule_3_steps": st3, "levels_last_step": hist, "ms_one_step_with_initial_forces": t1,
           "ms_three_steps": t3, "ms_per_dt_max_steady": steady,
           "active_fraction": upd / (n * 16), "particle_updates_per_s": upd / (steady * 1e-3),
           "tick_walks": ticks,
           "rebuild_before_every_walk": {"schedule_3_steps": rst3, "ms_per_dt_max_steady": steady_rb}}
    if shared_ms:
        out["ms_shared_16_smallest_steps"] = 16 * shared_ms
        out["speedup_vs_shared_smallest_steps"] = 16 * shared_ms / steady
        out["rebuild_before_every_walk"]["speedup_vs_shared_smallest_steps"] = 16 * shared_ms / steady_rb
    return out

def block_tick_walks(ctx, P, V, M, levels, theta, dt_min, reps=5):
    """The active walks of block time steps, one per due set that the last
    step's levels give (level >= r is due at the ticks aligned to dt_max/2^r):
    the walk's time (stage events, median of reps) against a full walk of the
    same tree, beside the shares of the particles evaluated and of the visited
    groups' work, work = particles x (n_pc + n_pp): the groups' whole lists are
    built (traversal) for every visited group, and only the active particles
    are evaluated.  Then the finest due set's walk on trees refitted after the
    particles drifted k ticks (k = 1, 2, 4) from the build, with its visited
    groups' interaction counts against the fresh tree's."""
    import numpy as np
    import torch
    from paper_1204_2280_amd import mibh
    ctx.forces(P, M, theta)
    ctx.sync()
    counts = ctx.export("counts").view(torch.int32).reshape(-1, 2).cpu().numpy().astype(np.int64)
    grp = mibh.Decoded.groups(ctx.export("groups"))
    perm = ctx.export("perm").cpu().numpy().view(np.uint32).astype(np.int64)
    lists = counts[:, 0] + counts[:, 1]
    gn = np.asarray(grp["count"], np.int64)
    gfirst = np.asarray(grp["first"], np.int64)
    total = float(np.sum(gn * lists))
    lev_sorted = levels.cpu().numpy()[perm]
    acc = torch.empty((P.shape[0], 3), dtype=torch.float32, device=P.device)
    pot = torch.empty((P.shape[0],), dtype=torch.float32, device=P.device)

    def walk_ms(fn):
        fn()
        ctx.sync()
        ctx.profile_begin(reps)
        for _ in range(reps):
            fn()
        return float(np.median([r["walk"] for r in ctx.profile_read()]))

    full_ms = walk_ms(lambda: ctx.compute_forces(theta, acc, pot))
    out = {"full_walk_ms": full_ms, "due_sets": []}
    for r in sorted(set(int(x) for x in np.unique(lev_sorted)), reverse=True):
        due_sorted = (lev_sorted >= r).astype(np.int64)
        csum = np.concatenate([[0], np.cumsum(due_sorted)])
        active_in_group = csum[gfirst + gn] - csum[gfirst]
        visited = active_in_group > 0
        mask = (levels >= r).to(torch.uint8)
        ms = walk_ms(lambda: ctx.compute_forces_active(theta, mask, acc, pot))
        out["due_sets"].append({
            "levels_due": f">= {r}", "particles_share": float(due_sorted.mean()),
            "groups_share": float(visited.mean()),
            "visited_groups_work_share": float(np.sum((gn * lists)[visited]) / total),
            "evaluated_work_share": float(np.sum(active_in_group * lists) / total),
            "walk_ms": ms, "walk_share": ms / full_ms})
    # refitted trees: the finest due set after k ticks of drift
    r = int(lev_sorted.max())
    mask = (levels >= r).to(torch.uint8)
    fresh_work = None
    P0 = P.clone()
    out["refit_drift"] = []
    for k in (0, 1, 2, 4):
        if k == 0:
            ctx.build_tree(P0, M)
        else:
            P.copy_(P0 + (k * dt_min) * V)
            ctx.refit(P, M)
        ctx.compute_multipoles()
        ms = walk_ms(lambda: ctx.compute_forces_active(theta, mask, acc, pot))
        c = ctx.export("counts").view(torch.int32).reshape(-1, 2).cpu().numpy().astype(np.int64)
        vis = np.zeros(len(gn), bool)
        csum = np.concatenate([[0], np.cumsum((lev_sorted >= r).astype(np.int64))])
        vis[(csum[gfirst + gn] - csum[gfirst]) > 0] = True
        work = float(np.sum((gn * (c[:, 0] + c[:, 1]))[vis]))
        if fresh_work is None:
            fresh_work = work
        out["refit_drift"].append({"ticks_since_build": k, "walk_ms": ms, "visited_work_vs_fresh": work / fresh_work})
    P.copy_(P0)
    return out


def bench_variant_neighbors(pos, mass, steps):
    """Neighbour search and SPH density on the benchmark sphere (tree of the
    force step; smoothing lengths from the analytic Plummer density for 64
    neighbours within 2h): milliseconds of neighbour counting, of CSR
    neighbour lists (counts, scan, fill) and of the density."""
    import torch
    from paper_1204_2280_amd import mibh, workloads
    n = len(mass)
    dev = torch.device("cuda", 0)
    P, M = torch.from_numpy(pos).to(dev), torch.from_numpy(mass).to(dev)
    h = torch.from_numpy(workloads.plummer_smoothing_lengths(pos, 64)).to(dev)
    r = 2.0 * h
    ctx = mibh.Context(n, device=dev)
    ctx.build_tree(P, M)
    ctx.compute_multipoles()

    def timed(fn):
        fn()
        ctx.sync()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(ctx.stream)
        for _ in range(steps):
            out = fn()
        b.record(ctx.stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps, out

    ms_count, cnt = timed(lambda: ctx.neighbor_count(r))
    total = int(cnt.sum())
    ms_list, _ = timed(lambda: ctx.neighbor_list(r, capacity=total))
    ms_rho, _ = timed(lambda: ctx.sph_density(h))
    del ctx
    return {"workload": f"plummer_n{n}_ngb64_support2h", "neighbours_per_particle": total / n,
            "ms_count": ms_count, "ms_list": ms_list, "ms_density": ms_rho,
            "neighbours_per_s_density": total / (ms_rho * 1e-3)}


def paper_sections(stage_ms):
    """The paper's five sections from the library's stage times."""
    return {"sorting": stage_ms["sorting"], "moving": stage_ms["moving"],
            "tree_construction": stage_ms["tree_construction"],
            "multipoles": stage_ms["multipoles"] + stage_ms["mac_prep"], "tree_traverse": stage_ms["walk"]}


def bench_config(pos, mass, theta, steps, warmup):
    """One force-step configuration: time per step, the paper's sections,
    interactions per particle and the walk's flop rate."""
    import numpy as np
    import torch
    from paper_1204_2280_amd import mibh
    n = len(mass)
    dev = torch.device("cuda", 0)
    p = torch.from_numpy(pos).to(dev)
    m = torch.from_numpy(mass).to(dev)
    ctx = mibh.Context(n, device=dev)
    acc = torch.empty((n, 3), dtype=torch.float32, device=dev)
    pot = torch.empty((n,), dtype=torch.float32, device=dev)
    for _ in range(warmup):
        ctx.forces(p, m, theta, acc, pot)
    ctx.sync()
    ctx.profile_begin(steps)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(ctx.stream)
    for _ in range(steps):
        ctx.forces(p, m, theta, acc, pot)
    b.record(ctx.stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    stages = ctx.profile_read()
    ctx.sync()
    st = ctx.stats()
    stage_ms = {k: float(np.mean([x[k] for x in stages])) for k in mibh.STAGES}
    flops = F_PC * st["sum_pc"] + F_PP * st["sum_pp"]
    del ctx
    return {"n": n, "theta": theta, "ms_per_step": ms, "particles_per_s": n / (ms * 1e-3),
            "paper_sections_ms": paper_sections(stage_ms),
            "interactions_per_particle": {"pc": st["sum_pc"] / n, "pp": st["sum_pp"] / n},
            "walk_tflops": flops / (stage_ms["walk"] * 1e-3) / 1e12}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1 << 22)
    ap.add_argument("--theta", type=float, default=0.75)
    ap.add_argument("--precision", choices=("plain", "kahan", "kahan_term"), default="plain")
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--walk-waves", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the Kahan and batched-ensemble variants")
    ap.add_argument("--copy-check-mib", type=int, default=0,
                    help="also run a plain device copy of this size (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the force step is single-GPU); --gpus {args.gpus} "
              "is not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1204_2280_amd import mibh, workloads

    n, theta = args.n, args.theta
    workload = f"plummer_n{n}_seed{args.seed}_theta{theta:g}_{args.precision}"
    log(f"[bench] workload {workload}")
    pos, _, mass = workloads.plummer(n, args.seed, with_velocities=False)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    p = torch.from_numpy(pos).to(dev)
    m = torch.from_numpy(mass).to(dev)
    ctx = mibh.Context(n, device=dev, precision={"plain": 0, "kahan": 1, "kahan_term": 2}[args.precision],
                       walk_waves=args.walk_waves)
    acc = torch.empty((n, 3), dtype=torch.float32, device=dev)
    pot = torch.empty((n,), dtype=torch.float32, device=dev)

    for _ in range(args.warmup):
        ctx.forces(p, m, theta, acc, pot)
    ctx.sync()
    log(f"[bench] warmup done ({args.warmup} steps)")

    ctx.profile_begin(args.steps)
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(ctx.stream)
    for _ in range(args.steps):
        ctx.forces(p, m, theta, acc, pot)
    end.record(ctx.stream)
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(end)
    stages = ctx.profile_read()
    ctx.sync()
    st = ctx.stats()
    log(f"[bench] timed {args.steps} steps: {total_ms:.2f} ms")

    ms_step = total_ms / args.steps
    stage_ms = {k: float(np.mean([s[k] for s in stages])) for k in mibh.STAGES}
    walk_ms = stage_ms["walk"]
    inter = st["sum_pc"] + st["sum_pp"]
    flops = F_PC * st["sum_pc"] + F_PP * st["sum_pp"]
    achieved = flops / (walk_ms * 1e-3) / 1e12
    sections = paper_sections(stage_ms)
    step_sums = sorted(sum(x[k] for k in mibh.STAGES) for x in stages)
    traffic = measured_traffic(workload)
    fma_tflops = fma_ceiling(dev)

    result = {
        "metric": "particles/s per full force step (build+walk), N=2^22 theta=0.75; interactions/s",
        "value": n * args.steps / (total_ms * 1e-3),
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload, "n": n, "theta": theta, "ncrit": 16, "group_cap": 64,
                   "precision": args.precision, "seed": args.seed, "multipoles": "f64",
                   "interactions": "f32"},
        "interactions_per_s": inter * args.steps / (total_ms * 1e-3),
        "interactions_per_particle": {"pc": st["sum_pc"] / n, "pp": st["sum_pp"] / n},
        "stage_ms": stage_ms,
        "paper_sections_ms": sections,
        "ms_per_step_stage_events": {"median": float(np.median(step_sums)), "min": step_sums[0]},
        "walk_share": walk_ms / ms_step,
        "hbm_stages": hbm_stages(stage_ms, n, st["ncells"]),
        "tree": {"ncells": st["ncells"], "ngroups": st["ngroups"], "nleaves": st["nleaves"],
                 "depth": st["depth"], "anchors": st["anchors"], "anchors_without_room": st["anchor_fallbacks"]},
        "roofline": {
            "kernel": "walk stage: k_walk_anchor + k_walk_claim + k_walk_prefix (shared anchor lists) + k_walk (group tree walk)",
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS,
            "traffic": traffic,
            "fma_measured": fma_tflops,
            "frac_of_fma_measured": achieved / fma_tflops,
            "flops_per_launch": flops,
            "walk_ms": walk_ms,
        },
    }
    if args.copy_check_mib > 0:
        nb = args.copy_check_mib << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        result["copy_check_bytes"] = nb
    if not args.no_variants:
        log("[bench] variant: opening angles 0.5 and 1.0")
        result["variant_theta"] = [bench_config(pos, mass, th, max(3, args.steps // 4), 1) for th in (0.5, 1.0)]
        log("[bench] variant: sections at N = 2^20")
        p20, _, m20 = workloads.plummer(1 << 20, 2, with_velocities=False)
        result["variant_sections_n1048576_seed2"] = bench_config(p20, m20, theta, args.steps, 2)
        log("[bench] variant: N = 2^24")
        p24, _, m24 = workloads.plummer(1 << 24, 9, with_velocities=False)
        result["variant_n16777216_seed9"] = bench_config(p24, m24, theta, max(3, args.steps // 4), 1)
        del p24, m24
        log("[bench] variant: kahan")
        result["variant_kahan"] = bench_variant_kahan(pos, mass, theta, max(3, args.steps // 4), 1)
        log("[bench] variant: learned estimator training")
        w16 = train_estimator(pos, mass, theta)
        log("[bench] variant: batched ensemble")
        result["variant_ensemble"], ens_out = bench_variant_ensemble(theta, max(3, args.steps // 4), 1, w16)
        log("[bench] variant: leapfrog driver")
        result["variant_leapfrog"] = bench_variant_leapfrog(n, args.seed, theta, 20)
        log("[bench] variant: block time steps")
        result["variant_block_steps"] = bench_variant_block_steps(
            n, args.seed, theta, result["variant_leapfrog"]["ms_per_step"])
        log("[bench] variant: neighbour search and SPH density")
        result["variant_neighbors"] = bench_variant_neighbors(pos, mass, 5)
        log("[bench] variant: queue order")
        result["variant_queue_order"] = bench_variant_queue_order(w16, theta, max(3, args.steps // 4))
        log("[bench] variants done")
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        result["cpu_baseline"] = cpu_baseline(pos, mass, theta)
        if not args.no_variants:
            log("[bench] cpu baseline: the ensemble")
            ce = cpu_baseline_ensemble(theta, ens_out)
            result["cpu_baseline"]["ensemble"] = ce
            cfg = result["variant_ensemble"]["graph_configs"]
            result["target_config"] = {
                "workload": result["variant_ensemble"]["workload"],
                "plain": {"what": "plain float32 accumulation, Morton queue, graph-replayed batched step",
                          "particles_per_s": cfg["plain_morton"]["particles_per_s"],
                          "acc_p99_vs_oracle": ce["acc_p99_vs_oracle"]["plain_morton"],
                          "pot_p99_vs_oracle": ce["pot_p99_vs_oracle"]["plain_morton"]},
                "target": {"what": "Kahan accumulation, learned-estimator queue order, graph-replayed batched step",
                           "particles_per_s": cfg["kahan_estimator"]["particles_per_s"],
                           "acc_p99_vs_oracle": ce["acc_p99_vs_oracle"]["kahan_estimator"],
                           "pot_p99_vs_oracle": ce["pot_p99_vs_oracle"]["kahan_estimator"]}}
        log("[bench] cpu baseline done")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
