"""Seeded synthetic inputs for the force step (test and benchmark plumbing).

This module produces particle sets only.  It holds none of the tree-code's
arithmetic (no keys, no tree, no multipoles, no forces) and imports nothing
from the rest of the package, so both the GPU path and the CPU oracle can be
fed from it without sharing any code with each other.

Workloads (the paper measures Plummer spheres of 2^15 .. 2^22 bodies at
theta = 0.75, Results section and the captions of Fig. 1 and Fig. 2):

* ``plummer(n, seed)``      Plummer (1915) sphere sampled with the method of
  Aarseth, Henon & Wielen (1974), in Henon units (G = M = 1, E = -1/4).
* ``hernquist(n, seed)``    Hernquist (1990) sphere, a = 1, M = 1, truncated
  at r = 50 (used by the ensemble workload; not in the paper).
* ``two_plummers(n_each)``  two Plummer spheres of 0.5 mass each at (+-5,0,0).
* ``ensemble(nsys, seed)``  uneven-N systems, N log-uniform in [2^12, 2^18].
* ``subsample(n, m, seed)`` m distinct indices by a partial Fisher-Yates.

Random numbers come from a counter-based splitmix64 stream (Steele, Lea &
Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014): draw
``i`` of stream ``s`` under seed ``seed`` is the splitmix64 output for state
``base(seed, s) + (i + 1) * gamma``; a uniform double in [0, 1) is the top 53
bits of that output times 2^-53.  All sampling is done in float64 and the
returned arrays are float32 (positions, velocities, masses), C-contiguous.
"""
from __future__ import annotations

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# stream identifiers (one independent counter sequence per sampled quantity)
S_RADIUS, S_COST, S_PHI, S_Q1, S_Q2, S_VCOST, S_VPHI, S_SIZE, S_PICK = range(1, 10)


def _mix(z: np.ndarray) -> np.ndarray:
    """splitmix64 output function, element-wise on uint64 (wrapping)."""
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64(x: int) -> int:
    """One splitmix64 step from state ``x``: returns the output for x + gamma."""
    s = np.array([x], dtype=np.uint64)
    with np.errstate(over="ignore"):
        return int(_mix(s + _GAMMA)[0])


def _base(seed: int, stream: int) -> np.uint64:
    s = np.array([(seed * 1000003 + stream) & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64)
    return _mix(s)[0]


def uniform(seed: int, stream: int, start: int, count: int) -> np.ndarray:
    """Draws start .. start+count-1 of (seed, stream) as float64 in [0, 1)."""
    idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = _mix(_base(seed, stream) + idx * _GAMMA)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def _isotropic(seed: int, s_cos: int, s_phi: int, n: int) -> np.ndarray:
    c = 2.0 * uniform(seed, s_cos, 0, n) - 1.0
    p = 2.0 * np.pi * uniform(seed, s_phi, 0, n)
    s = np.sqrt(np.maximum(0.0, 1.0 - c * c))
    return np.stack([s * np.cos(p), s * np.sin(p), c], axis=1)


def plummer(n: int, seed: int, *, with_velocities: bool = True):
    """Plummer sphere in Henon units: returns (pos f32[n,3], vel f32[n,3], mass f32[n]).

    Radii: r = 1/sqrt(X^(-2/3) - 1) with X ~ U[0, 0.999) (r < 38.7 before the
    Henon length scale).  Speeds: q * v_esc(r) with q drawn by rejection from
    the density q^2 (1 - q^2)^(7/2) (bounding box height 0.1).  Centre of mass
    position and velocity are removed in float64, then lengths are scaled by
    3 pi / 16 and speeds by sqrt(16 / (3 pi)); every mass is 1/n.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    x = 0.999 * uniform(seed, S_RADIUS, 0, n)
    with np.errstate(divide="ignore"):
        r = 1.0 / np.sqrt(np.power(x, -2.0 / 3.0) - 1.0)
    r[x == 0.0] = 0.0
    pos = r[:, None] * _isotropic(seed, S_COST, S_PHI, n)
    vel = np.zeros((n, 3), dtype=np.float64)
    if with_velocities:
        q = np.empty(n, dtype=np.float64)
        todo = np.arange(n)
        trial = 0
        while todo.size:
            q1 = uniform(seed, S_Q1, trial * n, n)[todo]
            q2 = 0.1 * uniform(seed, S_Q2, trial * n, n)[todo]
            ok = q2 < q1 * q1 * np.power(1.0 - q1 * q1, 3.5)
            q[todo[ok]] = q1[ok]
            todo = todo[~ok]
            trial += 1
        vesc = np.sqrt(2.0) * np.power(1.0 + r * r, -0.25)
        vel = (q * vesc)[:, None] * _isotropic(seed, S_VCOST, S_VPHI, n)
    pos -= pos.mean(axis=0)
    vel -= vel.mean(axis=0)
    pos *= 3.0 * np.pi / 16.0
    vel *= np.sqrt(16.0 / (3.0 * np.pi))
    mass = np.full(n, 1.0 / n, dtype=np.float32)
    return (np.ascontiguousarray(pos, dtype=np.float32),
            np.ascontiguousarray(vel, dtype=np.float32), mass)


def hernquist(n: int, seed: int):
    """Hernquist sphere (a = 1, M = 1) truncated at r = 50: (pos f32[n,3], mass f32[n]).

    Inverts M(<r) = r^2/(r+1)^2: r = sqrt(X)/(1 - sqrt(X)), X ~ U[0, (50/51)^2).
    The centre of mass is removed in float64.  Every mass is 1/n.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    x = (50.0 / 51.0) ** 2 * uniform(seed, S_RADIUS, 0, n)
    sx = np.sqrt(x)
    r = sx / (1.0 - sx)
    pos = r[:, None] * _isotropic(seed, S_COST, S_PHI, n)
    pos -= pos.mean(axis=0)
    mass = np.full(n, 1.0 / n, dtype=np.float32)
    return np.ascontiguousarray(pos, dtype=np.float32), mass


def two_plummers(n_each: int, seed_a: int = 5, seed_b: int = 6, separation: float = 10.0):
    """Two Henon-unit Plummer spheres of mass 0.5 each, centred at (-sep/2,0,0) and (+sep/2,0,0)."""
    pa, _, _ = plummer(n_each, seed_a, with_velocities=False)
    pb, _, _ = plummer(n_each, seed_b, with_velocities=False)
    pa = pa.astype(np.float64)
    pb = pb.astype(np.float64)
    pa[:, 0] -= 0.5 * separation
    pb[:, 0] += 0.5 * separation
    pos = np.ascontiguousarray(np.concatenate([pa, pb]), dtype=np.float32)
    mass = np.full(2 * n_each, 0.5 / n_each, dtype=np.float32)
    return pos, mass


def ensemble_sizes(nsys: int = 64, seed: int = 4, lo_log2: int = 12, hi_log2: int = 18):
    """N_k = floor(2^(lo + (hi - lo) u_k)) clamped to [2^lo, 2^hi]."""
    u = uniform(seed, S_SIZE, 0, nsys)
    n = np.floor(np.power(2.0, lo_log2 + (hi_log2 - lo_log2) * u)).astype(np.int64)
    return np.clip(n, 1 << lo_log2, 1 << hi_log2)


def ensemble(nsys: int = 64, seed: int = 4, lo_log2: int = 12, hi_log2: int = 18):
    """Concatenated uneven-N systems: first half Plummer, second half Hernquist.

    System k uses seed splitmix64(seed + k).  Returns (pos f32[sum N,3],
    mass f32[sum N], offsets int64[nsys+1]).
    """
    sizes = ensemble_sizes(nsys, seed, lo_log2, hi_log2)
    parts_p, parts_m = [], []
    for k in range(nsys):
        s = splitmix64(seed + k)
        if k < nsys // 2:
            p, _, m = plummer(int(sizes[k]), s, with_velocities=False)
        else:
            p, m = hernquist(int(sizes[k]), s)
        parts_p.append(p)
        parts_m.append(m)
    offsets = np.zeros(nsys + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    return (np.ascontiguousarray(np.concatenate(parts_p)),
            np.ascontiguousarray(np.concatenate(parts_m)), offsets)


def subsample(n: int, m: int, seed: int = 7) -> np.ndarray:
    """m distinct indices of range(n) by a partial Fisher-Yates shuffle (int64)."""
    m = min(m, n)
    a = np.arange(n, dtype=np.int64)
    u = uniform(seed, S_PICK, 0, m)
    for t in range(m):
        j = t + int(u[t] * (n - t))
        a[t], a[j] = a[j], a[t]
    return a[:m].copy()


def uniform_cube(n: int, seed: int, side: float = 1.0):
    """n particles uniform in [0, side)^3 with equal masses 1/n (edge-case tests)."""
    pos = np.stack([uniform(seed, s, 0, n) for s in (S_RADIUS, S_COST, S_PHI)], axis=1) * side
    return (np.ascontiguousarray(pos, dtype=np.float32),
            np.full(n, 1.0 / max(n, 1), dtype=np.float32))


def plummer_smoothing_lengths(pos, n_ngb: int = 64):
    """Smoothing lengths for SPH inputs on a Henon-unit Plummer sphere of
    len(pos) equal masses (total mass 1): h such that a sphere of radius 2h
    around the particle holds n_ngb particles on average under the analytic
    density rho(r) = 3/(4 pi a^3) (1 + r^2/a^2)^(-5/2), a = 3 pi/16 (the
    sphere is centred on the origin).  float32 [n]."""
    p = np.asarray(pos, np.float64)
    a = 3.0 * np.pi / 16.0
    r2 = np.sum(p * p, axis=1)
    rho = 3.0 / (4.0 * np.pi * a ** 3) * (1.0 + r2 / (a * a)) ** -2.5
    num = len(p) * rho
    return (0.5 * np.cbrt(3.0 * n_ngb / (4.0 * np.pi * num))).astype(np.float32)
