"""Limits of the force step: empty input is refused, and the largest size
tested, N = 2^24 (four times the benchmark's sphere), matches the oracle in
the benchmark's launch configuration: keys, permutation, cells, groups,
float64 multipoles and MAC data bit for bit; the interaction counts of
sampled group ranges bit for bit and their particles' accelerations and
potentials within 1e-5 at the 99th percentile."""
import numpy as np
import pytest

from gpu_helpers import TOL_P99, assert_multipoles_equal, assert_tree_equal, gpu_context, p99, rel_err, run_gpu
from paper_1204_2280_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_empty_input_is_refused():
    import torch
    from paper_1204_2280_amd import mibh
    ctx = gpu_context(100)
    p = torch.zeros((0, 3), dtype=torch.float32, device="cuda")
    m = torch.zeros((0,), dtype=torch.float32, device="cuda")
    with pytest.raises(mibh.MibhError) as e:
        ctx.build_tree(p, m)
    assert e.value.status == -1
    with pytest.raises(mibh.MibhError) as e:
        ctx.compute_forces(0.75)
    assert e.value.status == -4
    bc = gpu_context(100, max_systems=4)
    p2 = torch.rand((10, 3), dtype=torch.float32, device="cuda")
    m2 = torch.ones((10,), dtype=torch.float32, device="cuda")
    with pytest.raises(mibh.MibhError) as e:
        bc.build_tree_batch(p2, m2, [0, 4, 4, 10])  # the second system is empty
    assert e.value.status == -1


def test_largest_tested_size():
    import oracle
    n = 1 << 24
    pos, _, mass = W.plummer(n, 9, with_velocities=False)
    print(f"[gpu] N = {n}: oracle tree", flush=True)
    T = oracle.Tree(pos, mass)
    ctx = gpu_context(n)
    g = run_gpu(ctx, pos, mass, 0.75, exports=("keys", "perm", "cells", "groups", "counts", "multipoles",
                                                "delta", "mac"))
    assert_tree_equal(g, T)
    assert_multipoles_equal(g, T, 0.75)
    grp = T.groups()
    width = 128
    acc_g, pot_g, acc_o, pot_o = [], [], [], []
    for s in np.linspace(0, T.ngroups - width, 6).astype(np.int64):
        gb, ge = int(s), int(s) + width
        T.walk(0.75, groups=(gb, ge))
        npc, npp = T.counts()
        np.testing.assert_array_equal(g["counts"][gb:ge, 0], npc[gb:ge])
        np.testing.assert_array_equal(g["counts"][gb:ge, 1], npp[gb:ge])
        sacc, spot = T.sorted_forces()
        f0, f1 = grp["first"][gb], grp["first"][ge - 1] + grp["count"][ge - 1]
        idx = T.perm[f0:f1]
        acc_o.append(sacc[f0:f1])
        pot_o.append(spot[f0:f1])
        acc_g.append(g["acc"][idx])
        pot_g.append(g["pot"][idx])
    ea = rel_err(np.concatenate(acc_g), np.concatenate(acc_o))
    ep = rel_err(np.concatenate(pot_g), np.concatenate(pot_o))
    print(f"[gpu] N = {n}: {T.ncells} cells, {T.ngroups} groups, {ea.size} sampled particles, "
          f"acc p99 {p99(ea):.2e}, pot p99 {p99(ep):.2e}", flush=True)
    assert p99(ea) <= TOL_P99 and p99(ep) <= TOL_P99
