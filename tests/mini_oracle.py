"""Brute-force NumPy definitions used to pin the C oracle on tiny inputs.

These are declarative restatements (set definitions, exhaustive enumeration),
not a second copy of the oracle's procedures: the tree is the set of key
prefixes whose parent prefix holds more than ncrit particles; a cell is in a
group's particle-cell list iff it is accepted and every strict ancestor is
opened; the Morton order is checked with the most-significant-differing-bit
comparison of Chan (2002), which never builds a key.
"""
from __future__ import annotations

import numpy as np

KEY_BITS = 20


def msb(x: int) -> int:
    return x.bit_length() - 1


def morton_less(a, b) -> bool:
    """Z-order comparison of integer triples (x, y, z) without interleaving:
    the axis whose coordinates differ in the highest bit decides; on equal
    highest bits x outranks y outranks z (x is the most significant bit of
    every octal digit)."""
    best_axis, best_bit = None, -1
    for axis in range(3):
        d = int(a[axis]) ^ int(b[axis])
        if d == 0:
            continue
        m = msb(d)
        if m > best_bit:  # strictly greater: on ties keep the earlier axis
            best_axis, best_bit = axis, m
    if best_axis is None:
        return False
    return int(a[best_axis]) < int(b[best_axis])


def prefix(keys: np.ndarray, level: int) -> np.ndarray:
    return keys >> np.uint64(3 * (KEY_BITS - level))


def tree_cells(keys_sorted: np.ndarray, ncrit: int):
    """All cells as (level, first, count), ordered by level then first.

    A level-l prefix p is a cell iff l == 0, or its parent prefix p >> 3 is a
    cell holding more than ncrit particles with level l-1 < 20."""
    n = keys_sorted.shape[0]
    cells = [(0, 0, n)]
    split = {0: n > ncrit}  # prefix at current level -> does it split
    for lev in range(1, KEY_BITS + 1):
        pref = prefix(keys_sorted, lev)
        parent = prefix(keys_sorted, lev - 1)
        new_split = {}
        uniq, first, counts = np.unique(pref, return_index=True, return_counts=True)
        for p, f, c in zip(uniq, first, counts):
            if split.get(int(parent[f]), False):
                cells.append((lev, int(f), int(c)))
                new_split[int(p)] = c > ncrit and lev < KEY_BITS
        split = new_split
        if not split:
            break
    return sorted(cells)


def group_ranges(cells, gcap: int):
    """Groups as (first, count, level): cells with count <= gcap whose parent
    holds more than gcap (or the root), plus gcap-chunks of oversized level-20
    leaves.  Parents are found by containment, not by stored links."""
    out = []
    by_level = {}
    for (lev, f, c) in cells:
        by_level.setdefault(lev, []).append((f, c))
    for (lev, f, c) in cells:
        if lev == 0:
            parent_count = None
        else:
            parent_count = next(pc for (pf, pc) in by_level[lev - 1] if pf <= f < pf + pc)
        if parent_count is not None and parent_count <= gcap:
            continue
        if c <= gcap:
            out.append((f, c, lev))
        else:
            is_leaf = not any(pf == f for (pf, pc) in by_level.get(lev + 1, []))
            if is_leaf:
                for s in range(f, f + c, gcap):
                    out.append((s, min(gcap, f + c - s), lev))
    return sorted(out)


def mac_accept_f32(bmin, bmax, com32, r2open) -> bool:
    """The float32 predicate: squared distance from the box to the point,
    summed as (dx^2 + dy^2) + dz^2 with float32 rounding of each operation."""
    f = np.float32
    d = []
    for a in range(3):
        u = f(bmin[a]) - f(com32[a])
        v = f(com32[a]) - f(bmax[a])
        m = u if u > v else v
        d.append(m if m > f(0) else f(0))
    d2 = f(f(d[0] * d[0]) + f(d[1] * d[1])) + f(d[2] * d[2])
    return bool(d2 > f(r2open))


def group_sets(cells_arr, group, sposf, com32, r2open):
    """(PC, PP) index sets of one group by exhaustive enumeration over all
    cells: c is reachable iff every strict ancestor is opened; reachable
    accepted cells form PC, reachable opened leaves form PP."""
    lev, first, count, nchild = (cells_arr["level"], cells_arr["first"], cells_arr["count"],
                                 cells_arr["nchild"])
    gf, gc, gl = group
    pts = sposf[gf:gf + gc]
    bmin, bmax = pts.min(axis=0), pts.max(axis=0)
    nc = lev.shape[0]

    def opened(c):
        anc = first[c] <= gf < first[c] + count[c] and lev[c] <= gl
        return anc or not mac_accept_f32(bmin, bmax, com32[c], r2open[c])

    def ancestors(c):
        return [a for a in range(nc)
                if lev[a] < lev[c] and first[a] <= first[c] and first[c] + count[c] <= first[a] + count[a]]

    pc, pp = set(), set()
    for c in range(nc):
        if not all(opened(a) for a in ancestors(c)):
            continue
        if not opened(c):
            pc.add(c)
        elif nchild[c] == 0:
            pp.add(c)
    return pc, pp
