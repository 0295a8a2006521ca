"""Pins of the oracle's shared-time-step leapfrog (kick-drift-kick) against
closed forms and the integrator's own invariants.

* A single free particle moves on a straight line: x(t) = x0 + v0 t.
* Two equal masses on a circular orbit: the initial energies are the closed
  forms T = 1/8, W = -1/4; the orbit stays circular and returns to its start
  after one period.  On an eccentric orbit the energy error is second order
  in the step.
* Time reversal: k steps forward, velocities negated, k steps, velocities
  negated, gives back the initial state to float32 rounding (this fails for
  any first-order splitting, a missing or doubled half kick, or a kick and a
  drift taken in the wrong order).
"""
import numpy as np
import pytest

from paper_1204_2280_amd import workloads as W


@pytest.fixture(scope="module")
def lf(orc):
    from oracle import leapfrog
    return leapfrog


def test_free_particle_moves_on_a_line(lf):
    x0 = np.array([[0.25, -1.5, 3.0]], np.float32)
    v0 = np.array([[0.5, 0.125, -0.25]], np.float32)
    m = np.array([1.0], np.float32)
    x, v, a, p, log = lf.leapfrog(x0, v0, m, 0.75, 0.01, 100)
    assert np.all(a == 0) and np.all(p == 0)
    np.testing.assert_array_equal(v, v0)
    exact = x0.astype(np.float64) + v0.astype(np.float64) * 100 * float(np.float32(0.01))
    # one float32 rounding per step
    assert np.all(np.abs(x - exact) <= 100 * np.spacing(np.abs(exact).astype(np.float32)))


def _binary():
    x = np.array([[-0.5, 0.0, 0.0], [0.5, 0.0, 0.0]], np.float32)
    v = np.array([[0.0, -0.5, 0.0], [0.0, 0.5, 0.0]], np.float32)
    m = np.array([0.5, 0.5], np.float32)
    return x, v, m


def test_circular_binary(lf):
    x, v, m = _binary()
    period = 2 * np.pi  # radius 1/2, speed 1/2
    nstep = 400
    dt = period / nstep
    xf, vf, a, p, log = lf.leapfrog(x, v, m, 0.75, dt, nstep, log_every=10)
    T0, W0 = log[0, 1], log[0, 2]
    assert abs(T0 - 0.125) < 1e-15 and abs(W0 + 0.25) < 1e-15
    E = log[:, 1] + log[:, 2]
    drift = np.abs(E - E[0]) / abs(E[0])
    # leapfrog energy error ~ (omega dt)^2 / 8 for a circular orbit
    assert drift.max() < (dt ** 2) and drift.max() > 0
    sep = np.linalg.norm(xf[1].astype(np.float64) - xf[0].astype(np.float64))
    assert abs(sep - 1.0) < 1e-3
    # back near the start after one period (phase error O(dt^2))
    assert np.max(np.abs(xf.astype(np.float64) - x)) < 2e-3
    # momentum is conserved to rounding
    assert np.abs((m[:, None] * vf.astype(np.float64)).sum(0)).max() < 1e-7


def test_energy_error_is_second_order(lf):
    """Eccentric binary (apocentre 1, pericentre 0.22): the largest energy
    error over one orbit falls by 4 when the step is halved."""
    x, _, m = _binary()
    v = np.array([[0.0, -0.3, 0.0], [0.0, 0.3, 0.0]], np.float32)
    a_orbit = 1.0 / (2.0 * (1.0 - 0.5 * 0.6 ** 2))  # GM / (2 |specific energy|), GM = 1
    period = 2 * np.pi * np.sqrt(a_orbit ** 3)
    errs = []
    for nstep in (400, 800):
        _, _, _, _, log = lf.leapfrog(x, v, m, 0.75, period / nstep, nstep, log_every=1)
        E = log[:, 1] + log[:, 2]
        errs.append(np.abs(E - E[0]).max() / abs(E[0]))
    ratio = errs[0] / errs[1]
    assert 3.6 < ratio < 4.4, ratio


def test_time_reversal(lf):
    pos, vel, mass = W.plummer(64, 12)
    k = 20
    dt = 1.0 / 256
    x1, v1, _, _, _ = lf.leapfrog(pos, vel, mass, 1e-3, dt, k, eps2=0.01)
    x2, v2, _, _, _ = lf.leapfrog(x1, -v1, mass, 1e-3, dt, k, eps2=0.01)
    scale = np.abs(pos).max()
    assert np.max(np.abs(x2 - pos)) < 2e-5 * scale
    assert np.max(np.abs(-v2 - vel)) < 2e-5 * np.abs(vel).max()
    # a step without the closing half kick is not reversible
    from oracle.leapfrog import forces

    def euler_like(x, v, n):
        x = x.copy()
        v = v.copy()
        for _ in range(n):
            a, _ = forces(x, mass, 1e-3, eps2=0.01)
            v = (v + dt * a).astype(np.float32)
            x = (x + dt * v).astype(np.float32)
        return x, v
    y1, w1 = euler_like(pos, vel, k)
    y2, w2 = euler_like(y1, -w1, k)
    assert np.max(np.abs(y2 - pos)) > 100 * np.max(np.abs(x2 - pos))
