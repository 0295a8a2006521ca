"""Input generators against closed forms, and the hand-derived key fixture."""
import os

import numpy as np

from paper_1204_2280_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_golden_morton_keys(orc):
    rows = [l.split() for l in open(os.path.join(GOLDEN, "morton_keys.txt")) if l.strip() and l[0] != "#"]
    assert len(rows) >= 10
    for r in rows:
        lo = np.array([float(v) for v in r[0:3]], np.float32)
        k = int(r[3])
        x = np.array([float(v) for v in r[4:7]], np.float32)
        assert orc.key(x, lo, k) == int(r[7]), r


def test_plummer_closed_forms():
    n = 1 << 16
    pos, vel, mass = W.plummer(n, 1)
    assert pos.dtype == np.float32 and pos.shape == (n, 3) and mass.sum() == np.float32(1.0)
    a = 3 * np.pi / 16
    r = np.sort(np.linalg.norm(pos.astype(np.float64), axis=1))
    # enclosed mass M(r) = r^3 / (r^2 + a^2)^(3/2) (truncated at X < 0.999)
    frac = np.arange(1, n + 1) / n * 0.999
    Mr = r ** 3 / (r ** 2 + a ** 2) ** 1.5
    assert np.max(np.abs(Mr - frac)) < 1.5 / np.sqrt(n) * 2
    np.testing.assert_allclose(np.median(r), a / np.sqrt(2 ** (2 / 3) - 1), rtol=0.02)
    assert np.abs(pos.astype(np.float64).mean(0)).max() < 1e-6
    assert np.abs(vel.astype(np.float64).mean(0)).max() < 1e-6
    # kinetic energy 1/4 in Henon units (sampling noise ~ 1/sqrt(n))
    T = 0.5 * np.sum(mass * np.sum(vel.astype(np.float64) ** 2, axis=1))
    assert abs(T - 0.25) < 3 / np.sqrt(n)


def test_hernquist_closed_form():
    n = 1 << 15
    pos, mass = W.hernquist(n, 3)
    r = np.sort(np.linalg.norm(pos.astype(np.float64), axis=1))
    frac = np.arange(1, n + 1) / n * (50 / 51) ** 2
    Mr = r ** 2 / (r + 1) ** 2
    assert np.max(np.abs(Mr - frac)) < 3 / np.sqrt(n)
    assert r.max() < 51


def test_reproducible_and_seed_dependent():
    a = W.plummer(1000, 5)[0]
    b = W.plummer(1000, 5)[0]
    c = W.plummer(1000, 6)[0]
    np.testing.assert_array_equal(a, b)
    assert not np.array_equal(a, c)


def test_two_plummers_and_ensemble():
    pos, mass = W.two_plummers(4096)
    assert pos.shape == (8192, 3) and abs(mass.astype(np.float64).sum() - 1.0) < 1e-6
    assert pos[:4096, 0].mean() < -4 and pos[4096:, 0].mean() > 4
    sizes = W.ensemble_sizes(64, 4)
    assert sizes.min() >= 4096 and sizes.max() <= 262144
    p, m, off = W.ensemble(4, 4, 8, 10)
    assert off[-1] == p.shape[0] == m.shape[0] and off[0] == 0


def test_subsample_distinct():
    s = W.subsample(100000, 4096, 7)
    assert len(np.unique(s)) == 4096 and s.min() >= 0 and s.max() < 100000
