"""Parity at the benchmark's full size: N = 2^22 Plummer sphere (seed 3), in the
launch configuration the benchmark times (default parameters).

The oracle builds the whole tree (keys, permutation, cells, groups and float64
multipoles are compared in full) and walks every group: the interaction
counts of all groups must match bit for bit, and the accelerations and
potentials of all 4 194 304 particles to 1e-5 at the 99th percentile, for
theta in {0.5, 0.75, 1.0} with plain float32 accumulation, theta in
{0.5, 0.75} with Kahan compensation across list evaluations and theta = 0.75
with Kahan compensation of every term (same lists, so the same oracle walk).
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
    return pos, mass, T, ctx, {}


def _oracle_walk(T, cache, theta):
    """Counts and input-order forces of the oracle's walk of every group (cached per theta)."""
    if theta not in cache:
        print(f"[gpu] oracle walk of all {T.ngroups} groups, theta={theta}", flush=True)
        T.walk(theta)
        npc, npp = T.counts()
        acc, pot = T.forces()
        cache[theta] = (npc, npp, acc, pot)
    return cache[theta]


@pytest.mark.parametrize("theta,precision", [(0.75, 0), (0.75, 1), (0.75, 2), (0.5, 0), (0.5, 1), (1.0, 0)])
def test_full_size_parity(full, theta, precision):
    pos, mass, T, ctx0, cache = full
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
    npc, npp, acc_o, pot_o = _oracle_walk(T, cache, theta)
    np.testing.assert_array_equal(g["counts"][:, 0], npc)
    np.testing.assert_array_equal(g["counts"][:, 1], npp)
    ea = rel_err(g["acc"], acc_o)
    ep = rel_err(g["pot"], pot_o)
    print(f"[gpu] full size theta={theta} prec={precision}: all {ea.size} particles, acc p50 "
          f"{np.median(ea):.2e} p99 {p99(ea):.2e} max {ea.max():.2e}, pot p99 {p99(ep):.2e}", flush=True)
    assert ea.size == N
    assert p99(ea) <= TOL_P99 and p99(ep) <= TOL_P99
