"""Pins of the oracle's keys, sort, tree and groups (CPU only).

Every check compares the oracle with something it does not contain: worked
examples derived by hand from the key definition, a Morton comparison that
never interleaves bits, numpy's stable argsort, and declarative set
definitions of the tree and the groups enumerated by brute force.
"""
import numpy as np
import pytest

import mini_oracle as mo
from paper_1204_2280_amd import workloads as W


def test_root_cube_power_of_two_strictly_larger(orc):
    rng = np.random.default_rng(11)
    for scale in (1e-3, 0.7, 1.0, 3.0, 1000.0):
        pos = (rng.standard_normal((500, 3)) * scale).astype(np.float32)
        lo, k = orc.root_cube(pos)
        ext = max(float(pos[:, a].max()) - float(pos[:, a].min()) for a in range(3))
        L = 2.0 ** k
        assert L > ext and L / 2 <= ext, (scale, k, ext)
        np.testing.assert_array_equal(lo, pos.min(axis=0))
    # extent exactly a power of two: strictly larger cube
    pos = np.array([[0, 0, 0], [1, 0, 0]], np.float32)
    assert orc.root_cube(pos)[1] == 1
    # a single point: zero extent -> k = 0
    assert orc.root_cube(np.ones((1, 3), np.float32))[1] == 0


def test_keys_worked_examples(orc):
    lo = np.zeros(3, np.float32)
    # unit cube (k = 0): each axis has 2^20 cells of side 2^-20
    assert orc.key([0, 0, 0], lo, 0) == 0
    top = 1.0 - 2.0 ** -20
    assert orc.key([top, top, top], lo, 0) == 2 ** 60 - 1
    # half way along one axis sets the top bit of that axis only:
    # x -> bit 3*19+2, y -> bit 3*19+1, z -> bit 3*19
    assert orc.key([0.5, 0, 0], lo, 0) == 2 ** 59
    assert orc.key([0, 0.5, 0], lo, 0) == 2 ** 58
    assert orc.key([0, 0, 0.5], lo, 0) == 2 ** 57
    assert orc.key([0.25, 0.25, 0.25], lo, 0) == 2 ** 56 + 2 ** 55 + 2 ** 54
    # the smallest cell along z is bit 0, along x bit 2
    eps = 2.0 ** -20
    assert orc.key([0, 0, eps], lo, 0) == 1
    assert orc.key([eps, 0, 0], lo, 0) == 4
    # scale: cube of side 2^3 anchored at lo = (-4, -4, -4)
    lo2 = np.full(3, -4.0, np.float32)
    assert orc.key([0.0, -4.0, -4.0], lo2, 3) == 2 ** 59
    # a single-axis point sets only every third bit
    x = 0.6180339
    kx = orc.key([x, 0, 0], lo, 0)
    assert kx & ~sum(1 << (3 * b + 2) for b in range(20)) == 0
    q = int(np.floor(np.float64(np.float32(x)) * 2 ** 20))
    assert sum(((kx >> (3 * b + 2)) & 1) << b for b in range(20)) == q
    # the clamp: the maximum coordinate lands in the last cell
    pos = np.array([[0, 0, 0], [1, 1, 1]], np.float32)
    lo3, k3 = orc.root_cube(pos)
    assert k3 == 1 and orc.key([1, 1, 1], lo3, k3) == 2 ** 59 + 2 ** 58 + 2 ** 57


def test_key_order_matches_morton_comparison(orc):
    """Key order equals the Z-order comparison of the quantised coordinates."""
    rng = np.random.default_rng(5)
    pos = rng.random((300, 3)).astype(np.float32)
    T = orc.Tree(pos, np.full(300, 1 / 300, np.float32))
    lo, k = T.lo, T.k
    s = 2.0 ** (20 - k)
    q = np.minimum(np.floor((pos.astype(np.float64) - lo.astype(np.float64)) * s), 2 ** 20 - 1).astype(np.int64)
    keys = np.array([orc.key(p, lo, k) for p in pos], dtype=np.uint64)
    for _ in range(3000):
        i, j = rng.integers(0, 300, 2)
        assert (keys[i] < keys[j]) == mo.morton_less(q[i], q[j])


def test_sort_is_numpy_stable_argsort(orc):
    # include many duplicate keys: coarse grid of positions
    rng = np.random.default_rng(3)
    pos = (rng.integers(0, 4, (2000, 3)) * 0.25).astype(np.float32)
    mass = np.full(2000, 1 / 2000, np.float32)
    T = orc.Tree(pos, mass)
    keys_in = np.array([orc.key(p, T.lo, T.k) for p in pos], dtype=np.uint64)
    perm = np.argsort(keys_in, kind="stable")
    np.testing.assert_array_equal(T.perm, perm)
    np.testing.assert_array_equal(T.keys, keys_in[perm])


@pytest.mark.parametrize("case", ["plummer", "cube", "coincident", "line", "two_points", "tiny"])
def test_tree_and_groups_match_declarative_definition(orc, case):
    if case == "plummer":
        pos, _, mass = W.plummer(3000, 9, with_velocities=False)
    elif case == "cube":
        pos, mass = W.uniform_cube(1500, 4)
    elif case == "coincident":  # one level-20 leaf of 200 particles -> gcap chunks
        pos = np.tile(np.array([[0.3, -0.2, 0.1]], np.float32), (200, 1))
        pos = np.concatenate([pos, np.array([[1, 1, 1], [-1, 0, 0]], np.float32)])
        mass = np.full(202, 1 / 202, np.float32)
    elif case == "line":
        pos = np.zeros((700, 3), np.float32)
        pos[:, 0] = np.linspace(-1, 1, 700, dtype=np.float32)
        mass = np.full(700, 1 / 700, np.float32)
    elif case == "two_points":
        pos = np.array([[0, 0, 0], [1, 2, 3]], np.float32)
        mass = np.array([0.5, 0.5], np.float32)
    else:
        pos = np.array([[0.1, 0.2, 0.3]], np.float32)
        mass = np.array([1.0], np.float32)
    T = orc.Tree(pos, mass, ncrit=16, gcap=64)
    keys = T.keys
    cells = T.cells()
    got = sorted(zip(cells["level"].tolist(), cells["first"].tolist(), cells["count"].tolist()))
    assert got == mo.tree_cells(keys, 16)
    # breadth-first numbering: ordered by (level, first)
    order = list(zip(cells["level"].tolist(), cells["first"].tolist()))
    assert order == sorted(order)
    # children partition the parent range in octant order
    for c in range(T.ncells):
        if cells["nchild"][c] == 0:
            assert cells["count"][c] <= 16 or cells["level"][c] == 20
            continue
        assert cells["count"][c] > 16 and cells["level"][c] < 20
        ch = range(cells["child_first"][c], cells["child_first"][c] + cells["nchild"][c])
        assert cells["first"][ch[0]] == cells["first"][c]
        assert sum(cells["count"][x] for x in ch) == cells["count"][c]
        for a, b in zip(ch, ch[1:]):
            assert cells["first"][b] == cells["first"][a] + cells["count"][a]
        for x in ch:
            assert cells["parent"][x] == c and cells["level"][x] == cells["level"][c] + 1
            f = cells["first"][x]
            pre = keys[f:f + cells["count"][x]] >> np.uint64(3 * (20 - cells["level"][x]))
            assert np.all(pre == pre[0])
    g = T.groups()
    got_g = sorted(zip(g["first"].tolist(), g["count"].tolist(), g["level"].tolist()))
    assert got_g == mo.group_ranges(mo.tree_cells(keys, 16), 64)
    # groups partition [0, n) in order
    assert g["first"][0] == 0
    assert np.all(g["first"][1:] == g["first"][:-1] + g["count"][:-1])
    assert g["first"][-1] + g["count"][-1] == T.n
    assert np.all(g["count"] <= 64) and np.all(g["count"] >= 1)
    if case == "coincident":
        assert sorted(g["count"].tolist()) == [1, 1, 8, 64, 64, 64]


def test_tree_ncrit_variants(orc):
    pos, _, mass = W.plummer(2000, 21, with_velocities=False)
    for ncrit, gcap in ((8, 32), (16, 64), (32, 128), (1, 1)):
        T = orc.Tree(pos, mass, ncrit=ncrit, gcap=gcap)
        got = sorted(zip(*[T.cells()[k].tolist() for k in ("level", "first", "count")]))
        assert got == mo.tree_cells(T.keys, ncrit)
        gg = T.groups()
        got_g = sorted(zip(gg["first"].tolist(), gg["count"].tolist(), gg["level"].tolist()))
        assert got_g == mo.group_ranges(mo.tree_cells(T.keys, ncrit), gcap)


def test_invalid_inputs_rejected(orc):
    pos = np.zeros((4, 3), np.float32)
    mass = np.ones(4, np.float32)
    bad = pos.copy()
    bad[2, 1] = np.nan
    with pytest.raises(orc.OracleError):
        orc.Tree(bad, mass)
    with pytest.raises(orc.OracleError):
        orc.Tree(pos, -mass)
    with pytest.raises(orc.OracleError):
        orc.Tree(pos, mass, ncrit=65, gcap=64)
    T = orc.Tree(pos, mass)
    with pytest.raises(orc.OracleError):
        T.walk(0.0)
