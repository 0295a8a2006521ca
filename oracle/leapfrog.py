"""Shared-time-step leapfrog of the oracle (TEST INFRASTRUCTURE ONLY).

Only the test-suite may import this module; the GPU library shares no code
with it.

The paper integrates every step on the GPU without host traffic
(Introduction; Results section) but names no integrator.  The reading taken
is the kick-drift-kick leapfrog: forces at the initial positions, then per
step

    v <- v + (dt/2) a(x),   x <- x + dt v,   v <- v + (dt/2) a(x).

The state is float32, as the library's interface fixes it; every update is
evaluated in float64 from the float32 values and rounded to float32 once.
Forces are the oracle tree-code's (float64, the same keys, tree and MAC as
the force step), and the energy log holds (t, T, W) from the oracle's
float64 energy sums.
"""
from __future__ import annotations

import numpy as np

from . import Tree, energy


def forces(pos32, mass32, theta, eps2=0.0, G=1.0, nthreads=0, ncrit=16, gcap=64):
    """Tree-code acceleration and potential (float64) at float32 positions."""
    t = Tree(pos32, mass32, ncrit, gcap)
    t.walk(theta, eps2, G, nthreads=nthreads)
    a, p = t.forces()
    return a.copy(), p.copy()


def leapfrog(pos, vel, mass, theta, dt, nsteps, log_every=0, eps2=0.0, G=1.0, nthreads=0, ncrit=16, gcap=64):
    """Returns (pos f32, vel f32, acc f64, pot f64, log f64[k, 3]) after nsteps steps."""
    x = np.array(pos, dtype=np.float32).reshape(-1, 3)
    v = np.array(vel, dtype=np.float32).reshape(-1, 3)
    m = np.array(mass, dtype=np.float32).reshape(-1)
    step = float(np.float32(dt))          # the step is a float32 argument
    half = float(np.float32(0.5) * np.float32(dt))
    a, p = forces(x, m, theta, eps2, G, nthreads, ncrit, gcap)
    log = []

    def record(s):
        T, W = energy(m, p, v)
        log.append((s * step, T, W))

    if log_every > 0:
        record(0)
    for s in range(1, nsteps + 1):
        v = (v.astype(np.float64) + half * a).astype(np.float32)
        x = (x.astype(np.float64) + step * v.astype(np.float64)).astype(np.float32)
        a, p = forces(x, m, theta, eps2, G, nthreads, ncrit, gcap)
        v = (v.astype(np.float64) + half * a).astype(np.float32)
        if log_every > 0 and s % log_every == 0:
            record(s)
    return x, v, a, p, np.array(log, dtype=np.float64).reshape(-1, 3)
