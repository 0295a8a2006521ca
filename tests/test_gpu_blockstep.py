"""Block time steps on the GPU (mibh_block_run) against the oracle's.

* One level with a rebuild every tick is the GPU's shared-step leapfrog, bit
  for bit.
* A softened 2^12 Plummer sphere over two steps of dt_max = 1/16 with five
  levels (32 ticks, refits and rebuilds by the work trigger): the same
  schedule (ticks, rebuilds, particle updates, groups walked) and levels as
  the oracle; positions and velocities within 1e-5 at p99 (1e-3 at most) of
  the component scale, energies within 1e-6 (both sides keep float32 state;
  they differ by the float32 interactions, <= 1e-5 per force at p99, and one
  rounding per update).
"""
import numpy as np
import pytest

from gpu_helpers import gpu_context
from paper_1204_2280_amd import workloads as W

pytestmark = pytest.mark.gpu


def _t(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def test_one_level_rebuilding_every_tick_is_the_leapfrog():
    pos, vel, mass = W.plummer(3000, 18)
    a = gpu_context(len(mass))
    P, V, M = _t(pos), _t(vel), _t(mass)
    a.block_run(P, V, M, 0.75, 1 / 64, 0, 0.1, 0.01, 6, rebuild_tol=-1.0)
    b = gpu_context(len(mass))
    P2, V2 = _t(pos), _t(vel)
    b.leapfrog(P2, V2, M, 0.75, 1 / 64, 6)
    a.sync()
    b.sync()
    assert bool((P == P2).all()) and bool((V == V2).all())


@pytest.mark.parametrize("tol", [0.05, -1.0])  # refits with a work-growth trigger; a rebuild before every walk
def test_block_steps_match_oracle(orc, tol):
    from oracle import blockstep
    n, theta, eps2 = 1 << 12, 0.75, 1e-4
    dt_max, R, eta, eps, nbig = 1 / 16, 4, 0.1, 0.1, 2
    pos, vel, mass = W.plummer(n, 13)
    ctx = gpu_context(n, eps2=eps2)
    P, V, M = _t(pos), _t(vel), _t(mass)
    print(f"[gpu] block steps n={n} R={R} nbig={nbig} rebuild tolerance {tol}", flush=True)
    acc, pot, lev, st, log = ctx.block_run(P, V, M, theta, dt_max, R, eta, eps, nbig, rebuild_tol=tol)
    ctx.sync()
    x, v, a, p, olev, ost, olog = blockstep.block_run(pos, vel, mass, theta, dt_max, R, eta, eps, nbig, tol=tol,
                                                       eps2=eps2)
    print(f"[gpu] schedule gpu {st} oracle {ost}; levels {np.bincount(olev, minlength=R + 1)}", flush=True)
    assert st == ost
    np.testing.assert_array_equal(lev.cpu().numpy(), olev)
    gx, gv = P.cpu().numpy().astype(np.float64), V.cpu().numpy().astype(np.float64)
    ex = np.linalg.norm(gx - x, axis=1) / np.abs(pos).max()
    ev = np.linalg.norm(gv - v, axis=1) / np.abs(vel).max()
    print(f"[gpu] block steps pos diff p99 {np.percentile(ex, 99):.2e} max {ex.max():.2e}; "
          f"vel diff p99 {np.percentile(ev, 99):.2e} max {ev.max():.2e}", flush=True)
    assert np.percentile(ex, 99) <= 1e-5 and ex.max() <= 1e-3
    assert np.percentile(ev, 99) <= 1e-5 and ev.max() <= 1e-3
    np.testing.assert_array_equal(log[:, 0], olog[:, 0])
    Eg, Eo = log[:, 1] + log[:, 2], olog[:, 1] + olog[:, 2]
    print(f"[gpu] energies gpu {Eg} oracle {Eo}", flush=True)
    assert np.all(np.abs(Eg - Eo) <= 1e-6 * np.abs(Eo))


def test_block_run_argument_errors():
    import torch
    from paper_1204_2280_amd import mibh
    ctx = gpu_context(100)
    P = torch.rand((50, 3), device="cuda")
    V = torch.zeros((50, 3), device="cuda")
    M = torch.ones(50, device="cuda")
    for kw in ({"max_level": 21}, {"max_level": -1}, {"dt_max": 0.0}, {"eta": -1.0}, {"eps": float("nan")}):
        args = dict(dt_max=0.1, max_level=2, eta=0.1, eps=0.1)
        args.update(kw)
        with pytest.raises(mibh.MibhError):
            ctx.block_run(P, V, M, 0.75, args["dt_max"], args["max_level"], args["eta"], args["eps"], 1)


def test_block_run_stops_when_the_state_turns_nonfinite():
    """A NaN velocity makes one position NaN at the first drift; the first
    tick with a due particle refits a tree with it, its walk does nothing, and
    the driver stops there with ENONFINITE.  A clean run on the same context
    afterwards returns normally."""
    import torch
    from paper_1204_2280_amd import mibh
    pos, vel, mass = W.plummer(2000, 6)
    bad = vel.copy()
    bad[5, 2] = np.nan
    ctx = gpu_context(len(mass), eps2=1e-4)
    M = _t(mass)
    print("[gpu] block run with a NaN velocity, R=2, 1 step", flush=True)
    with pytest.raises(mibh.MibhError) as ei:
        ctx.block_run(_t(pos), _t(bad), M, 0.75, 1 / 16, 2, 0.1, 0.1, 1)
    assert ei.value.status == -6
    P = _t(pos)
    ctx.block_run(P, _t(vel), M, 0.75, 1 / 16, 2, 0.1, 0.1, 1)
    assert bool(torch.isfinite(P).all())
