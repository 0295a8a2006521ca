"""Shared-time-step leapfrog on the GPU against the oracle's leapfrog.

* kick_drift: each update is one float32 fused multiply-add; the reference is
  the float64 expression rounded once to float32, equal except where float64
  rounding before the final rounding moves a tie (at most 1 ulp).
* A 32-step run of a 2^12 Plummer sphere (theta 0.75, dt = 1/128): both
  sides keep float32 state, so they differ by the force differences (float32
  interactions vs float64, <= 1e-5 at p99 per step) and one float32 rounding
  per update, amplified by the dynamics over 32 steps: the tolerance is
  1e-5 at p99 and 1e-3 at most on positions and velocities (relative to the
  component scale), and 1e-6 on every logged energy.
"""
import numpy as np
import pytest

from gpu_helpers import gpu_context
from paper_1204_2280_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_kick_drift_is_one_rounding_per_update():
    import torch
    rng = np.random.default_rng(5)
    n = 100003
    x = rng.standard_normal((n, 3)).astype(np.float32)
    v = rng.standard_normal((n, 3)).astype(np.float32)
    a = (rng.standard_normal((n, 3)) * 10).astype(np.float32)
    ctx = gpu_context(n)
    X, V, A = (torch.from_numpy(t.copy()).cuda() for t in (x, v, a))
    dtk, dtd = np.float32(0.0078125), np.float32(0.015625)
    ctx.kick_drift(X, V, A, float(dtk), float(dtd))
    ctx.sync()
    v1 = (v.astype(np.float64) + float(dtk) * a.astype(np.float64)).astype(np.float32)
    x1 = (x.astype(np.float64) + float(dtd) * v1.astype(np.float64)).astype(np.float32)
    gv, gx = V.cpu().numpy(), X.cpu().numpy()
    assert np.all(np.abs(gv - v1) <= np.spacing(np.abs(v1)))
    assert np.all(np.abs(gx - x1) <= np.spacing(np.abs(x1)))
    assert np.mean(gv == v1) > 0.999 and np.mean(gx == x1) > 0.999
    # a kick alone leaves the positions untouched
    ctx.kick_drift(X, V, A, float(dtk), 0.0)
    ctx.sync()
    np.testing.assert_array_equal(X.cpu().numpy(), gx)


def test_leapfrog_matches_oracle(orc):
    import torch
    from oracle import leapfrog as lf
    n, steps, dt, theta = 1 << 12, 32, 1.0 / 128, 0.75
    pos, vel, mass = W.plummer(n, 11)
    ctx = gpu_context(n)
    P, V, M = (torch.from_numpy(t.copy()).cuda() for t in (pos, vel, mass))
    print(f"[gpu] leapfrog n={n} steps={steps}", flush=True)
    acc, pot, log = ctx.leapfrog(P, V, M, theta, dt, steps, log_every=8)
    ctx.sync()
    x, v, a, p, olog = lf.leapfrog(pos, vel, mass, theta, dt, steps, log_every=8)
    gx, gv = P.cpu().numpy().astype(np.float64), V.cpu().numpy().astype(np.float64)
    ex = np.linalg.norm(gx - x, axis=1) / np.abs(pos).max()
    ev = np.linalg.norm(gv - v, axis=1) / np.abs(vel).max()
    print(f"[gpu] leapfrog pos diff p99 {np.percentile(ex, 99):.2e} max {ex.max():.2e}; "
          f"vel diff p99 {np.percentile(ev, 99):.2e} max {ev.max():.2e}", flush=True)
    assert np.percentile(ex, 99) <= 1e-5 and ex.max() <= 1e-3
    assert np.percentile(ev, 99) <= 1e-5 and ev.max() <= 1e-3
    assert log.shape == olog.shape == (steps // 8 + 1, 3)
    np.testing.assert_array_equal(log[:, 0], olog[:, 0])
    Eg, Eo = log[:, 1] + log[:, 2], olog[:, 1] + olog[:, 2]
    print(f"[gpu] energies gpu {Eg} oracle {Eo}", flush=True)
    assert np.all(np.abs(Eg - Eo) <= 1e-6 * np.abs(Eo))
    # the forces returned are those of the final positions
    ra = np.linalg.norm(acc.cpu().numpy() - a, axis=1) / np.linalg.norm(a, axis=1)
    assert np.percentile(ra, 99) <= 1e-4


def test_leapfrog_argument_errors():
    import torch
    from paper_1204_2280_amd import mibh
    ctx = gpu_context(100)
    P = torch.zeros((10, 3), device="cuda")
    V = torch.zeros((10, 3), device="cuda")
    M = torch.ones(10, device="cuda")
    with pytest.raises(mibh.MibhError):
        ctx.leapfrog(P, V, M, 0.75, float("nan"), 2)
    with pytest.raises(mibh.MibhError):
        ctx.leapfrog(P, V, M, 0.75, 0.01, -1)
    with pytest.raises(ValueError):
        ctx.kick_drift(P, V[:5], P, 0.1, 0.1)


def test_leapfrog_reports_a_state_that_turns_nonfinite_mid_run():
    """A NaN velocity makes one position NaN at the first drift; the walks
    after that build do nothing, and the driver must say so (ENONFINITE) even
    though later builds reset the per-build flags.  The context stays usable:
    a clean run on it afterwards returns normally."""
    import torch
    from paper_1204_2280_amd import mibh
    pos, vel, mass = W.plummer(2000, 5)
    bad = vel.copy()
    bad[17, 0] = np.nan
    ctx = gpu_context(len(mass))
    M = torch.from_numpy(mass).cuda()
    P, V = torch.from_numpy(pos.copy()).cuda(), torch.from_numpy(bad).cuda()
    print("[gpu] leapfrog with a NaN velocity, 3 steps, no energy log", flush=True)
    with pytest.raises(mibh.MibhError) as ei:
        ctx.leapfrog(P, V, M, 0.75, 1 / 64, 3)
    assert ei.value.status == -6
    P, V = torch.from_numpy(pos.copy()).cuda(), torch.from_numpy(vel.copy()).cuda()
    ctx.leapfrog(P, V, M, 0.75, 1 / 64, 3)
    ctx.sync()
    assert bool(torch.isfinite(P).all())
