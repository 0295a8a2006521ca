"""Neighbour search and SPH density of the oracle (TEST INFRASTRUCTURE ONLY).

Only the test-suite may import this module; the GPU library shares no code
with it.  The paper's Discussion notes that the same tree serves neighbour
search and smoothed particle hydrodynamics; it gives no definitions, so the
readings are:

* neighbours of particle i (gather form): every j (i itself included) with
  d2 <= r_i * r_i, where d = x_j - x_i and d2 = (dx*dx + dy*dy) + dz*dz, all
  in float32 with each operation rounded (so any implementation decides each
  pair the same way);
* SPH density: rho_i = sum over the neighbours within 2 h_i of m_j W(r_ij, h_i)
  with the cubic-spline kernel of Monaghan & Lattanzio (1985),
  W(r, h) = 1/(pi h^3) * (1 - 3/2 q^2 + 3/4 q^3) for q = r/h < 1,
  1/(pi h^3) * (2 - q)^3 / 4 for 1 <= q < 2, and 0 beyond; evaluated here in
  float64 on the neighbour sets of the float32 predicate with r_i = 2 h_i.

Brute force over all pairs, in blocks of rows.
"""
from __future__ import annotations

import numpy as np


def _d2_block(pos32, rows):
    """float32 squared distances from particles `rows` to every particle, each
    operation rounded: (dx*dx + dy*dy) + dz*dz with d = x_j - x_i."""
    x = pos32[None, :, :]
    xi = pos32[rows][:, None, :]
    d = (x - xi).astype(np.float32)
    sq = (d * d).astype(np.float32)
    return ((sq[..., 0] + sq[..., 1]).astype(np.float32) + sq[..., 2]).astype(np.float32)


def neighbor_lists(pos, radius, rows=None, block=256):
    """Sorted neighbour indices of each particle in `rows` (all when None)."""
    p = np.ascontiguousarray(pos, np.float32).reshape(-1, 3)
    r = np.ascontiguousarray(radius, np.float32).reshape(-1)
    rows = np.arange(len(p)) if rows is None else np.asarray(rows)
    out = []
    for b in range(0, len(rows), block):
        rb = rows[b:b + block]
        d2 = _d2_block(p, rb)
        r2 = (r[rb] * r[rb]).astype(np.float32)
        for k in range(len(rb)):
            out.append(np.nonzero(d2[k] <= r2[k])[0])
    return out


def neighbor_counts(pos, radius, rows=None, block=256):
    return np.array([len(x) for x in neighbor_lists(pos, radius, rows, block)], np.int64)


def kernel_w(r, h):
    """Cubic spline W(r, h) in float64."""
    r = np.asarray(r, np.float64)
    h = np.asarray(h, np.float64)
    q = r / h
    s = 1.0 / (np.pi * h ** 3)
    return np.where(q < 1.0, s * (1.0 - 1.5 * q * q + 0.75 * q * q * q),
                    np.where(q < 2.0, s * 0.25 * (2.0 - q) ** 3, 0.0))


def sph_density(pos, mass, h, rows=None, block=256):
    """(rho f64, neighbour counts) for `rows` (all when None), support 2 h_i."""
    p = np.ascontiguousarray(pos, np.float32).reshape(-1, 3)
    m = np.ascontiguousarray(mass, np.float32).reshape(-1).astype(np.float64)
    hh = np.ascontiguousarray(h, np.float32).reshape(-1)
    rows = np.arange(len(p)) if rows is None else np.asarray(rows)
    support = (np.float32(2.0) * hh).astype(np.float32)
    lists = neighbor_lists(p, support, rows, block)
    p64 = p.astype(np.float64)
    rho = np.zeros(len(rows))
    for k, i in enumerate(rows):
        j = lists[k]
        r = np.linalg.norm(p64[j] - p64[i], axis=1)
        rho[k] = np.sum(m[j] * kernel_w(r, float(hh[i])))
    return rho, np.array([len(x) for x in lists], np.int64)
