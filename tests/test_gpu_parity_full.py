"""Parity at the benchmark's full size: N = 2^22 Plummer sphere (seed 3), in the
launch configuration the benchmark times (default parameters).

The oracle builds the whole tree (keys, permutation, cells, groups and float64
multipoles are compared in full) and walks sampled ranges of groups; the
interaction counts of those groups must match bit for bit and their particles'
accelerations and potentials to 1e-5 at the 99th percentile.
"""
import numpy as np
import pytest

from gpu_helpers import TOL_P99, assert_multipoles_equal, assert_tree_equal, gpu_context, p99, rel_err, run_gpu
from paper_1204_2280_amd import workloads as W

pytestmark = pytest.mark.gpu

N = 1 << 22


@pytest.fixture(scope="module")
def full():
    import oracle
    pos, _, mass = W.plummer(N, 3, with_velocities=False)
    print("[gpu] full-size oracle tree", flush=True)
    T = oracle.Tree(pos, mass)
    ctx = gpu_context(N)
    return pos, mass, T, ctx


def _sample_ranges(ngroups, k=8, width=160):
    starts = np.linspace(0, ngroups - width, k).astype(np.int64)
    return [(int(s), int(s) + width) for s in starts]


@pytest.mark.parametrize("theta,precision", [(0.75, 0), (0.5, 0), (1.0, 0), (0.75, 1)])
def test_full_size_parity(full, theta, precision):
    pos, mass, T, ctx0 = full
    ctx = ctx0 if precision == 0 else gpu_context(N, precision=precision)
    print(f"[gpu] full size theta={theta} precision={precision}", flush=True)
    exports = ("keys", "perm", "cells", "groups", "counts", "multipoles", "delta", "mac") \
        if (theta, precision) == (0.75, 0) else ("counts", "mac")
    g = run_gpu(ctx, pos, mass, theta, exports=exports)
    if "cells" in g:
        assert_tree_equal(g, T)
        assert_multipoles_equal(g, T, theta)
    else:
        np.testing.assert_array_equal(g["mac"][:, 3], T.mac_prep(theta)["r2open"])
    grp = T.groups()
    acc_g, pot_g, acc_o, pot_o = [], [], [], []
    for (gb, ge) in _sample_ranges(T.ngroups):
        T.walk(theta, groups=(gb, ge))
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
    print(f"[gpu] full size theta={theta} prec={precision}: {ea.size} particles, acc p99 {p99(ea):.2e} "
          f"max {ea.max():.2e}, pot p99 {p99(ep):.2e}", flush=True)
    assert p99(ea) <= TOL_P99 and p99(ep) <= TOL_P99
