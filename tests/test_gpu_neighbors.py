"""Neighbour search and SPH density on the GPU against the oracle's brute
force (the same float32 pair predicate, so counts and lists are compared
exactly; densities within 1e-5 at p99: float32 sums of positive terms).

Cases: a Plummer sphere with smoothing lengths from its analytic density,
random points with random radii, a zero radius (self and coincident points),
a clump of coincident points, one particle, and the 2^22 benchmark sphere on
a sample of particles.
"""
import numpy as np
import pytest

from gpu_helpers import gpu_context, p99
from paper_1204_2280_amd import workloads as W

pytestmark = pytest.mark.gpu


def _t(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _ctx(pos, mass):
    ctx = gpu_context(len(mass))
    ctx.build_tree(_t(pos), _t(mass))
    ctx.compute_multipoles()
    return ctx


def _cases():
    rng = np.random.default_rng(21)
    pos, _, mass = W.plummer(8192, 22, with_velocities=False)
    yield "plummer", pos, mass, 2.0 * W.plummer_smoothing_lengths(pos, 32)
    p = rng.random((5000, 3)).astype(np.float32)
    yield "random", p, np.full(5000, 2e-4, np.float32), (0.02 + 0.08 * rng.random(5000)).astype(np.float32)
    q = np.concatenate([rng.random((300, 3)), np.repeat(rng.random((1, 3)), 200, 0)]).astype(np.float32)
    yield "clump", q, np.full(500, 1e-3, np.float32), np.full(500, 0.05, np.float32)
    yield "zero_radius", q, np.full(500, 1e-3, np.float32), np.zeros(500, np.float32)
    yield "single", np.array([[0.5, 0.5, 0.5]], np.float32), np.ones(1, np.float32), np.ones(1, np.float32)


@pytest.mark.parametrize("case", [c[0] for c in _cases()])
def test_counts_and_lists_match_oracle(orc, case):
    from oracle import neighbors as nb
    name, pos, mass, r = next(c for c in _cases() if c[0] == case)
    print(f"[gpu] neighbours {name} n={len(mass)}", flush=True)
    ctx = _ctx(pos, mass)
    R = _t(r)
    cnt = ctx.neighbor_count(R).cpu().numpy().astype(np.int64)
    ref = nb.neighbor_lists(pos, r)
    np.testing.assert_array_equal(cnt, [len(x) for x in ref])
    c2, off, idx = ctx.neighbor_list(R)
    c2, off, idx = c2.cpu().numpy(), off.cpu().numpy().astype(np.int64), idx.cpu().numpy()
    np.testing.assert_array_equal(c2, cnt)
    np.testing.assert_array_equal(np.diff(off), cnt)
    assert off[0] == 0 and off[-1] == len(idx)
    for i in range(len(mass)):
        np.testing.assert_array_equal(np.sort(idx[off[i]:off[i + 1]]), ref[i])


def test_few_waves_drain_every_queue(orc):
    """Neighbour search on a grid of 3 persistent waves (fewer than the 8 per-XCD group queues):
    the same counts and lists as the oracle."""
    from oracle import neighbors as nb
    name, pos, mass, r = next(c for c in _cases() if c[0] == "random")
    ctx = gpu_context(len(mass), walk_waves=3)
    ctx.build_tree(_t(pos), _t(mass))
    ctx.compute_multipoles()
    R = _t(r)
    cnt = ctx.neighbor_count(R).cpu().numpy().astype(np.int64)
    ref = nb.neighbor_lists(pos, r)
    np.testing.assert_array_equal(cnt, [len(x) for x in ref])
    c2, off, idx = ctx.neighbor_list(R)
    off, idx = off.cpu().numpy().astype(np.int64), idx.cpu().numpy()
    for i in range(len(mass)):
        np.testing.assert_array_equal(np.sort(idx[off[i]:off[i + 1]]), ref[i])


def test_list_capacity_overflow():
    from paper_1204_2280_amd import mibh
    pos, _, mass = W.plummer(2000, 23, with_velocities=False)
    ctx = _ctx(pos, mass)
    R = _t(np.full(2000, 0.3, np.float32))
    total = int(ctx.neighbor_count(R).sum())
    with pytest.raises(mibh.MibhError):
        ctx.neighbor_list(R, capacity=total - 1)
    _, off, idx = ctx.neighbor_list(R, capacity=total)
    assert len(idx) == total


@pytest.mark.parametrize("case", ["plummer", "random", "clump"])
def test_density_matches_oracle(orc, case):
    from oracle import neighbors as nb
    name, pos, mass, r = next(c for c in _cases() if c[0] == case)
    h = (0.5 * r).astype(np.float32)
    ctx = _ctx(pos, mass)
    rho, cnt = ctx.sph_density(_t(h))
    rho, cnt = rho.cpu().numpy().astype(np.float64), cnt.cpu().numpy().astype(np.int64)
    ref, rcnt = nb.sph_density(pos, mass, h)
    np.testing.assert_array_equal(cnt, rcnt)
    err = np.abs(rho - ref) / ref
    print(f"[gpu] density {name}: p99 rel err {p99(err):.2e}, max {err.max():.2e}", flush=True)
    assert p99(err) <= 1e-5


def test_full_size_sample(orc):
    from oracle import neighbors as nb
    n = 1 << 22
    pos, _, mass = W.plummer(n, 3, with_velocities=False)
    h = W.plummer_smoothing_lengths(pos, 64)
    rows = W.subsample(n, 256, 7)
    ctx = _ctx(pos, mass)
    print("[gpu] neighbours at 2^22", flush=True)
    rho, cnt = ctx.sph_density(_t(h))
    rho, cnt = rho.cpu().numpy().astype(np.float64), cnt.cpu().numpy().astype(np.int64)
    ref, rcnt = nb.sph_density(pos, mass, h, rows=rows, block=8)
    np.testing.assert_array_equal(cnt[rows], rcnt)
    err = np.abs(rho[rows] - ref) / ref
    print(f"[gpu] 2^22 sample: neighbours {rcnt.mean():.1f} on average, density p99 rel err {p99(err):.2e}",
          flush=True)
    assert p99(err) <= 1e-5
