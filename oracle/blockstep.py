"""Block time steps of the oracle (TEST INFRASTRUCTURE ONLY).

Only the test-suite may import this module; the GPU library shares no code
with it.

The paper's block time steps (Results and Discussion sections) walk only the
particles that are due, refit the tree between rebuilds and rebuild it when
the walk slows down; it names no scheme.  The reading taken, step by step:

* particle i steps with dt_max / 2^r_i, r_i in 0..R, the smallest r with
  dt_max / 2^r <= eta sqrt(eps / |a_i|) (r = 0 for a = 0), taken in float64
  as the smallest r with 16^r >= dt_max^4 |a|^2 / (eta^4 eps^2);
* a clock ticks in dt_max / 2^R; every particle drifts every tick; at tick s
  the particles whose 2^(R - r_i) divides s are due; if any is, the tree is
  refitted (or rebuilt), the groups holding a due particle are walked (each
  with its whole box, so its lists are those of a full walk), the due particles
  get new accelerations and potentials (the others keep theirs), and each due
  particle gets its closing half kick (old level), a new level (at least
  R - (trailing zeros of s), so that its next step starts on its own grid)
  and its opening half kick;
* after each walk, the walked groups' work count * (1 + n_pc + n_pp) is
  summed against their work at their first walk after the last build (the
  initial walk sets every group's); when
  it exceeds (1 + tol) times that, the next tick rebuilds (tol < 0: every
  tick rebuilds).

State is float32 as in the library's interface; each update is evaluated in
float64 from float32 values and rounded once.  The energy log holds
(t, T, W) at every multiple of dt_max, between the closing and the opening
kicks.
"""
from __future__ import annotations

import numpy as np

from . import Tree, energy


def level_of(acc, dt_max, eta, eps, R, rmin=0):
    """Step level per particle from float64 accelerations [n, 3]."""
    a = np.asarray(acc, np.float64)
    a2 = (a[:, 0] * a[:, 0] + a[:, 1] * a[:, 1]) + a[:, 2] * a[:, 2]
    dt = float(np.float32(dt_max))
    q = ((dt * dt) * (dt * dt)) * a2 / (((eta * eta) * (eta * eta)) * (eps * eps))
    r = np.zeros(len(a2), np.int64)
    p = np.ones(len(a2))
    for _ in range(R):
        up = (a2 > 0) & (p < q)
        r += up
        p = np.where(up, p * 16.0, p)
    return np.maximum(r, rmin)


def _aligned(tick, R):
    if tick == 0:
        return 0
    tz = (tick & -tick).bit_length() - 1
    return 0 if tz >= R else R - tz


def block_run(pos, vel, mass, theta, dt_max, R, eta, eps, nbig, tol=0.25, eps2=0.0, G=1.0, nthreads=0,
              ncrit=16, gcap=64):
    """Returns (pos f32, vel f32, acc f64, pot f64, levels, stats dict, log f64[nbig + 1, 3])."""
    x = np.array(pos, dtype=np.float32).reshape(-1, 3)
    v = np.array(vel, dtype=np.float32).reshape(-1, 3)
    m = np.array(mass, dtype=np.float32).reshape(-1)
    n = len(m)
    eta = float(np.float32(eta))
    eps = float(np.float32(eps))
    tol = float(np.float32(tol))
    half_max = float(np.float32(0.5) * np.float32(dt_max))
    dt_min = float(np.ldexp(np.float32(dt_max), -R))
    nsub = 1 << R

    def kick(a, lev, sel):
        h = np.ldexp(half_max, -lev[sel])[:, None]
        v[sel] = (v[sel].astype(np.float64) + h * a[sel]).astype(np.float32)

    T = Tree(x, m, ncrit, gcap)
    T.walk(theta, eps2, G, nthreads=nthreads)
    a, p = (t.copy() for t in T.forces())
    npc, npp = T.counts()
    gref = T.groups()["count"] * (1 + npc + npp)  # the first walk sets every group's reference work
    stats = {"substeps": 0, "rebuilds": 0, "active_updates": 0, "groups_walked": 0}
    log = [(0.0, *energy(m, p, v))]
    lev = level_of(a, dt_max, eta, eps, R)
    if nbig > 0:
        kick(a, lev, np.ones(n, bool))
    rebuild = tol < 0  # negative: every tick rebuilds, the first one too
    for big in range(nbig):
        for tick in range(1, nsub + 1):
            x = (x.astype(np.float64) + dt_min * v.astype(np.float64)).astype(np.float32)
            due = (tick % (1 << (R - lev))) == 0
            stats["substeps"] += 1
            if not due.any():  # nobody is due: the particles only drift (a pending rebuild waits)
                continue
            if rebuild:
                T = Tree(x, m, ncrit, gcap)
                gref = np.zeros(T.ngroups, np.int64)
                stats["rebuilds"] += 1
                rebuild = False
            else:
                T.refit(x, m)
            g = T.groups()
            sdue = due[T.perm]
            walk = np.array([k for k in range(T.ngroups) if sdue[g["first"][k]:g["first"][k] + g["count"][k]].any()],
                            np.int64)
            T.walk_groups(theta, walk, eps2, G, nthreads=nthreads)
            ta, tp = T.forces()
            # the walked groups' lists serve only their due particles
            a[due] = ta[due]
            p[due] = tp[due]
            npc, npp = T.counts()
            now = g["count"][walk] * (1 + npc[walk] + npp[walk])
            ref = gref[walk]
            known = ref > 0
            work_now, work_ref = int(now[known].sum()), int(ref[known].sum())
            gref[walk[~known]] = now[~known]
            stats["active_updates"] += int(due.sum())
            stats["groups_walked"] += len(walk)
            rebuild = tol < 0 or (work_ref > 0 and work_now > (1.0 + tol) * work_ref)
            if tick == nsub:
                kick(a, lev, due)
                log.append(((big + 1) * float(np.float32(dt_max)), *energy(m, p, v)))
                if big + 1 < nbig:
                    lev = level_of(a, dt_max, eta, eps, R, 0)
                    kick(a, lev, due)
            else:
                kick(a, lev, due)
                new = level_of(a, dt_max, eta, eps, R, _aligned(tick, R))
                lev = np.where(due, new, lev)
                kick(a, lev, due)
    return x, v, a, p, lev, stats, np.array(log, np.float64)
