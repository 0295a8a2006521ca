"""Pins of the oracle's multipoles, MAC, walk and forces (CPU only).

Closed forms (two point masses, the Plummer potential), limits (theta -> 0
gives direct summation), convergence order of the expansion, invariants
(every particle is counted exactly once in each list, momentum), and a
brute-force enumeration of the interaction sets on tiny inputs.
"""
import numpy as np
import pytest

import mini_oracle as mo
from paper_1204_2280_amd import workloads as W


def _direct_s(pos, mass, idx):
    """Direct sum in numpy for a few targets, float64, skipping coincident pairs."""
    p = pos.astype(np.float64)
    m = mass.astype(np.float64)
    acc = np.zeros((len(idx), 3))
    pot = np.zeros(len(idx))
    for t, i in enumerate(idx):
        d = p - p[i]
        r2 = np.sum(d * d, axis=1)
        ok = r2 > 0
        rinv = np.zeros_like(r2)
        rinv[ok] = 1.0 / np.sqrt(r2[ok])
        acc[t] = np.sum((m * rinv ** 3)[:, None] * d, axis=0)
        pot[t] = -np.sum(m * rinv)
    return acc, pot


def test_direct_summation_matches_numpy(orc):
    pos, _, mass = W.plummer(700, 2, with_velocities=False)
    a, p = orc.direct(pos, mass)
    idx = np.arange(0, 700, 37)
    a2, p2 = _direct_s(pos, mass, idx)
    np.testing.assert_allclose(a[idx], a2, rtol=1e-12, atol=0)
    np.testing.assert_allclose(p[idx], p2, rtol=1e-12, atol=0)


def test_root_multipoles_closed_form(orc):
    n = 4096
    pos, _, mass = W.plummer(n, 4, with_velocities=False)
    T = orc.Tree(pos, mass)
    mp = T.multipoles()
    # masses are 2^-12: every partial sum is exact
    assert mp["M"][0] == 1.0
    x = pos.astype(np.float64)
    m = mass.astype(np.float64)
    com = (m[:, None] * x).sum(0) / m.sum()
    np.testing.assert_allclose(mp["com"][0], com, rtol=0, atol=1e-15)
    d = x - mp["com"][0]
    S = np.array([np.sum(m * d[:, a] * d[:, b]) for a, b in ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))])
    np.testing.assert_allclose(mp["S"][0], S, rtol=1e-11, atol=1e-15)


def test_every_cell_moments_equal_direct_sums(orc):
    """Parallel-axis shifts reproduce the second moments of each cell's own particles."""
    pos, _, mass = W.plummer(3000, 8, with_velocities=False)
    mass = mass * np.linspace(0.5, 1.5, 3000).astype(np.float32)  # unequal masses
    T = orc.Tree(pos, mass)
    mp = T.multipoles()
    c = T.cells()
    x = pos[T.perm].astype(np.float64)
    m = mass[T.perm].astype(np.float64)
    pairs = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))
    for cell in range(T.ncells):
        f, n = c["first"][cell], c["count"][cell]
        xs, ms = x[f:f + n], m[f:f + n]
        M = ms.sum()
        com = (ms[:, None] * xs).sum(0) / M
        np.testing.assert_allclose(mp["M"][cell], M, rtol=1e-13)
        np.testing.assert_allclose(mp["com"][cell], com, rtol=0, atol=1e-13)
        d = xs - com
        S = np.array([np.sum(ms * d[:, a] * d[:, b]) for a, b in pairs])
        scale = max(np.abs(S).max(), 1e-300)
        np.testing.assert_allclose(mp["S"][cell], S, rtol=0, atol=1e-10 * scale)
        Q = mp["Q"][cell]
        assert abs(Q[0] + Q[1] + Q[2]) <= 1e-12 * max(1e-300, np.abs(Q).max())
        np.testing.assert_allclose(Q[3:], 3 * S[3:], rtol=1e-12, atol=1e-14 * scale)
        # geometric centre from the cell's own particles: corner = lo + floor((x - lo)/l) l
        side = 2.0 ** (T.k - c["level"][cell])
        lo = T.lo.astype(np.float64)
        q = np.floor((xs[0] - lo) / side)
        centre = lo + (q + 0.5) * side
        assert np.all(xs >= centre - side / 2) and np.all(xs < centre + side / 2)
        np.testing.assert_allclose(mp["delta"][cell], np.linalg.norm(mp["com"][cell] - centre),
                                   rtol=1e-12, atol=1e-15 * side)
        assert mp["delta"][cell] <= np.sqrt(3) / 2 * side * (1 + 1e-12)


def _probe_setup(cluster_pos, cluster_mass, probe_pos):
    """Cluster inside the level-1 cell [0,2)^3 of a root cube [0,4)^3 (fixed by
    two massless anchors), 64 massless probes in the cell above it (z >= 2).
    The root holds more than 64 particles, so the cluster's cell and the probe
    cell are separate groups; the probes' forces are exactly the particle-cell
    terms of the cells they accept (all other sources are massless)."""
    anchors = np.array([[0, 0, 0], [3.9, 3.9, 3.9]])
    pos = np.concatenate([anchors, cluster_pos, probe_pos]).astype(np.float32)
    mass = np.concatenate([[0, 0], cluster_mass, np.zeros(len(probe_pos))]).astype(np.float32)
    return pos, mass


def _cluster_leaf(T, ncl):
    c = T.cells()
    leaf = [i for i in range(T.ncells) if c["level"][i] == 1 and c["count"][i] == ncl + 1]
    assert len(leaf) == 1 and c["nchild"][leaf[0]] == 0
    return leaf[0]


def _probes_accept(T, leaf, theta, nprobe):
    g = T.groups()
    seen = 0
    for gi in range(T.ngroups):
        f = g["first"][gi]
        members = T.perm[f:f + g["count"][gi]]
        if members.min() >= T.n - nprobe:
            pc, _ = T.group_lists(gi, theta)
            assert leaf in pc.tolist()
            seen += g["count"][gi]
    assert seen == nprobe


def test_two_mass_quadrupole_closed_form(orc):
    """Masses m at C +- s z: to quadrupole order, on the axis,
    phi = -(2m/r)(1 + s^2/r^2) and a_z = -(2m/r^2)(1 + 3 s^2/r^2); the octupole
    vanishes by symmetry, so the expansion is exact to O((s/r)^4)."""
    m, s = 0.25, 0.01
    C = np.array([1.0, 1.0, 1.0])
    cluster = np.array([C + [0, 0, s], C - [0, 0, s]])
    r = 1.5 + 0.02 * np.arange(64)
    probes = C + np.stack([np.zeros(64), np.zeros(64), r], axis=1)
    pos, mass = _probe_setup(cluster, [m, m], probes)
    T = orc.Tree(pos, mass)
    theta = 2.0
    leaf = _cluster_leaf(T, 2)
    _probes_accept(T, leaf, theta, 64)
    T.walk(theta)
    acc, pot = T.forces()
    mp = T.multipoles()
    zc = pos[2:4, 2].astype(np.float64)
    s_eff = 0.5 * (zc[0] - zc[1])
    np.testing.assert_allclose(mp["Q"][leaf][2], 4 * m * s_eff ** 2, rtol=1e-12)
    np.testing.assert_allclose(mp["Q"][leaf][0], -2 * m * s_eff ** 2, rtol=1e-12)
    rr = pos[4:, 2].astype(np.float64) - mp["com"][leaf][2]
    phi_cf = -(2 * m / rr) * (1 + s_eff ** 2 / rr ** 2)
    az_cf = -(2 * m / rr ** 2) * (1 + 3 * s_eff ** 2 / rr ** 2)
    np.testing.assert_allclose(pot[4:], phi_cf, rtol=1e-9)
    np.testing.assert_allclose(acc[4:, 2], az_cf, rtol=1e-9)
    assert np.max(np.abs(acc[4:, :2])) < 1e-12
    # the quadrupole term is really there: the monopole alone is off by 3 s^2/r^2 ~ 1e-4
    assert np.min(np.abs(acc[4:, 2] + 2 * m / rr ** 2) / np.abs(az_cf)) > 1e-5


def test_expansion_error_falls_as_third_power(orc):
    """Random 15-particle cluster of size s: the relative error of the
    particle-cell force vs direct summation falls as s^3 with the quadrupole
    (it would fall as s^2 with a wrong or missing quadrupole term)."""
    rng = np.random.default_rng(17)
    C = np.array([1.0, 1.0, 1.0])
    unit = rng.uniform(-1, 1, (15, 3))
    cm = rng.uniform(0.5, 1.5, 15) / 15
    probes = np.stack([rng.uniform(0.2, 1.8, 64), rng.uniform(0.2, 1.8, 64),
                       rng.uniform(2.3, 3.8, 64)], axis=1)
    errs = []
    for s in (0.16, 0.08, 0.04, 0.02):
        pos, mass = _probe_setup(C + s * unit, cm, probes)
        T = orc.Tree(pos, mass)
        leaf = _cluster_leaf(T, 15)
        _probes_accept(T, leaf, 2.0, 64)
        T.walk(2.0)
        acc, _ = T.forces()
        ad, _ = orc.direct(pos, mass, targets=np.arange(17, 81))
        e = np.linalg.norm(acc[17:] - ad, axis=1) / np.linalg.norm(ad, axis=1)
        errs.append(np.median(e))
    slopes = np.diff(np.log(errs)) / np.log(0.5)
    assert np.all(slopes > 2.6) and np.all(slopes < 3.6), (errs, slopes)


def test_mac_equality_opens(orc):
    """Two masses symmetric about the centre (1,1,1) of the level-1 cell of side
    2 give delta = 0 and, at theta = 2, r_open = 1 exactly.  A probe group whose
    box is exactly at distance 1 from the centre of mass must open the cell;
    moving the nearest probe up by one float32 step must accept it."""
    cluster = np.array([[1, 1, 1.25], [1, 1, 0.75]])
    for bump, accepted in ((0.0, False), (2.0 ** -22, True)):
        probes = np.stack([np.full(64, 1.0), np.full(64, 1.0), 2.0 + bump + 0.01 * np.arange(64)], axis=1)
        pos, mass = _probe_setup(cluster, [0.5, 0.5], probes)
        T = orc.Tree(pos, mass)
        leaf = _cluster_leaf(T, 2)
        assert T.multipoles()["delta"][leaf] == 0.0
        assert T.mac_prep(2.0)["r2open"][leaf] == 1.0
        g = T.groups()
        gi = [i for i in range(T.ngroups) if T.perm[g["first"][i]] >= 4][0]
        pc, pp = T.group_lists(gi, 2.0)
        assert (leaf in pc.tolist()) == accepted and (leaf in pp.tolist()) == (not accepted)


def test_ancestors_of_the_group_are_always_opened(orc):
    """At a very large theta the root cell itself would pass the distance test
    for a far probe group; it must still be opened because it contains the
    group, so every particle is counted exactly once."""
    cluster = np.array([[1, 1, 1.25], [1, 1, 0.75]])
    rng = np.random.default_rng(2)
    probes = rng.uniform(2.2, 3.8, (64, 3))
    pos, mass = _probe_setup(cluster, [0.5, 0.5], probes)
    T = orc.Tree(pos, mass)
    c = T.cells()
    for theta in (2.0, 100.0):
        for gi in range(T.ngroups):
            pc, pp = T.group_lists(gi, theta)
            assert 0 not in pc.tolist()
            assert c["count"][pc].sum() + c["count"][pp].sum() == T.n


def test_theta_to_zero_is_direct_summation(orc):
    pos, _, mass = W.plummer(3000, 12, with_velocities=False)
    T = orc.Tree(pos, mass)
    T.walk(1e-6)
    acc, pot = T.forces()
    npc, npp = T.counts()
    assert np.all(npc == 0) and np.all(npp == 3000)
    ad, pd = orc.direct(pos, mass)
    np.testing.assert_allclose(acc, ad, rtol=1e-11, atol=1e-12 * np.abs(ad).max())
    np.testing.assert_allclose(pot, pd, rtol=1e-12)


@pytest.mark.parametrize("theta", [0.5, 0.75, 1.0])
def test_every_particle_counted_once(orc, theta):
    pos, _, mass = W.plummer(20000, 13, with_velocities=False)
    T = orc.Tree(pos, mass)
    c = T.cells()
    for gi in range(0, T.ngroups, 37):
        pc, pp = T.group_lists(gi, theta)
        assert c["count"][pc].sum() + c["count"][pp].sum() == T.n
    T.walk(theta)
    npc, npp = T.counts()
    assert npc.min() > 0 and npp.min() >= T.groups()["count"].min()


def test_interaction_sets_match_brute_force(orc):
    for seed, n, theta in ((1, 300, 0.75), (2, 500, 0.5), (3, 400, 1.0), (4, 200, 1.3)):
        pos, _, mass = W.plummer(n, seed, with_velocities=False)
        T = orc.Tree(pos, mass)
        mac = T.mac_prep(theta)
        cells = T.cells()
        g = T.groups()
        sposf = pos[T.perm]
        for gi in range(T.ngroups):
            pc, pp = T.group_lists(gi, theta)
            epc, epp = mo.group_sets(cells, (g["first"][gi], g["count"][gi], g["level"][gi]), sposf,
                                     mac["com32"], mac["r2open"])
            assert set(pc.tolist()) == epc and set(pp.tolist()) == epp


def test_mac_data_definition(orc):
    """r2open is (l/theta + delta)^2 rounded once to float32; com32 is com rounded."""
    pos, _, mass = W.plummer(2000, 6, with_velocities=False)
    T = orc.Tree(pos, mass)
    mp = T.multipoles()
    lev = T.cells()["level"]
    for theta in (0.5, 0.75, 1.0):
        mac = T.mac_prep(theta)
        l = np.ldexp(1.0, T.k - lev)
        ro = l / np.float64(np.float32(theta)) + mp["delta"]
        np.testing.assert_array_equal(mac["r2open"], (ro * ro).astype(np.float32))
        np.testing.assert_array_equal(mac["com32"], mp["com"].astype(np.float32))


def test_momentum_and_accuracy_ordering(orc):
    n = 32768
    pos, vel, mass = W.plummer(n, 1)
    T = orc.Tree(pos, mass)
    sub = W.subsample(n, 512, 7)
    ad, pd = orc.direct(pos, mass, targets=sub)
    p99 = []
    for theta in (0.5, 0.75, 1.0):
        T.walk(theta)
        acc, pot = T.forces()
        e = np.linalg.norm(acc[sub] - ad, axis=1) / np.linalg.norm(ad, axis=1)
        p99.append(np.percentile(e, 99))
        if theta == 0.75:
            m = mass.astype(np.float64)
            mom = np.linalg.norm((m[:, None] * acc).sum(0)) / np.sum(m * np.linalg.norm(acc, axis=1))
            assert mom < 1e-3
            assert np.percentile(e, 99) < 2e-2
    assert p99[0] < p99[1] < p99[2]


def test_plummer_potential_and_virial(orc):
    n = 32768
    pos, vel, mass = W.plummer(n, 1)
    T = orc.Tree(pos, mass)
    T.walk(0.5)
    acc, pot = T.forces()
    a = 3 * np.pi / 16
    r = np.linalg.norm(pos.astype(np.float64), axis=1)
    phi = -1.0 / np.sqrt(r * r + a * a)
    rms = np.sqrt(np.mean(((pot - phi) / np.abs(phi)) ** 2))
    assert rms < 5 / np.sqrt(n)
    Tk, Wp = orc.energy(mass, pot, vel)
    assert abs(Wp + 0.5) < 3 / np.sqrt(n)
    assert abs(Tk - 0.25) < 3 / np.sqrt(n)
    assert abs((Tk + Wp) + 0.25) < 3 / np.sqrt(n)


def test_softening_and_G_scale(orc):
    pos, _, mass = W.plummer(1000, 14, with_velocities=False)
    T = orc.Tree(pos, mass)
    T.walk(1e-6, eps2=0.01, G=2.0)
    acc, pot = T.forces()
    ad, pd = orc.direct(pos, mass, eps2=0.01, G=2.0)
    np.testing.assert_allclose(acc, ad, rtol=1e-11, atol=1e-12 * np.abs(ad).max())
    # softened direct sum by hand for one particle
    x = pos.astype(np.float64)
    d = x - x[5]
    r2 = np.sum(d * d, axis=1)
    ok = r2 > 0
    a5 = 2.0 * np.sum((mass[ok] / (r2[ok] + 0.01) ** 1.5)[:, None] * d[ok], axis=0)
    np.testing.assert_allclose(acc[5], a5, rtol=1e-12)
