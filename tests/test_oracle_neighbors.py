"""Pins of the oracle's neighbour search and SPH density.

* Counts equal a k-d tree query of the library (scipy) on a lattice whose
  coordinates and squared distances are exact in float32 and whose radius
  matches no lattice distance, and on random points (where a pair at the
  boundary is improbable).
* A zero radius finds the particle itself and the points coincident with it.
* The cubic spline integrates to one over its support, is continuous at
  q = 1 and q = 2 and has W(0) = 1/(pi h^3).
* On a cubic lattice of spacing s and mass m the density away from the edges
  is m / s^3 to within the kernel's lattice error (< 1% for h = 1.2 s).
"""
import numpy as np
import pytest

scipy_spatial = pytest.importorskip("scipy.spatial")


@pytest.fixture(scope="module")
def nb(orc):
    from oracle import neighbors
    return neighbors


def _lattice(k, s):
    g = np.arange(k, dtype=np.float64) * s
    return np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3).astype(np.float32)


def test_counts_match_kdtree_on_exact_lattice(nb):
    pos = _lattice(12, 0.25)
    r = np.full(len(pos), 0.6, np.float32)
    got = nb.neighbor_counts(pos, r)
    ref = np.array([len(x) for x in scipy_spatial.cKDTree(pos.astype(np.float64)).query_ball_point(
        pos.astype(np.float64), 0.6)])
    np.testing.assert_array_equal(got, ref)
    # an interior point: itself and the shells at 0.25 (6), 0.354 (12), 0.433 (8), 0.5 (6), 0.559 (24)
    assert got.max() == 1 + 6 + 12 + 8 + 6 + 24


def test_counts_match_kdtree_on_random_points(nb):
    rng = np.random.default_rng(11)
    pos = rng.random((3000, 3)).astype(np.float32)
    r = (0.05 + 0.1 * rng.random(3000)).astype(np.float32)
    got = nb.neighbor_counts(pos, r)
    tree = scipy_spatial.cKDTree(pos.astype(np.float64))
    ref = np.array([len(tree.query_ball_point(pos[i].astype(np.float64), float(r[i]))) for i in range(3000)])
    np.testing.assert_array_equal(got, ref)
    lists = nb.neighbor_lists(pos, r, rows=[5, 17])
    for k, i in enumerate([5, 17]):
        np.testing.assert_array_equal(lists[k], np.sort(tree.query_ball_point(pos[i].astype(np.float64), float(r[i]))))


def test_zero_radius_finds_self_and_coincident(nb):
    pos = np.array([[0, 0, 0], [1, 1, 1], [0, 0, 0], [2, 0, 0]], np.float32)
    got = nb.neighbor_counts(pos, np.zeros(4, np.float32))
    np.testing.assert_array_equal(got, [2, 1, 2, 1])


def test_kernel_normalisation_and_continuity(nb):
    h = 0.7
    r = np.linspace(0.0, 2.0 * h, 200001)
    integrand = 4.0 * np.pi * r * r * nb.kernel_w(r, h)
    total = np.sum(0.5 * (integrand[1:] + integrand[:-1]) * np.diff(r))
    assert abs(total - 1.0) < 1e-9
    eps = 1e-9
    for q in (1.0, 2.0):
        assert abs(nb.kernel_w(q * h - eps, h) - nb.kernel_w(q * h + eps, h)) < 1e-6
    assert abs(nb.kernel_w(0.0, h) - 1.0 / (np.pi * h ** 3)) < 1e-15
    assert nb.kernel_w(2.0 * h, h) == 0.0


def test_lattice_density(nb):
    s, k = 0.25, 14
    pos = _lattice(k, s)
    m = np.full(len(pos), 0.5, np.float32)
    h = np.full(len(pos), 1.2 * s, np.float32)
    centre = np.nonzero(np.all((pos >= 5 * s) & (pos <= 8 * s), axis=1))[0]
    rho, cnt = nb.sph_density(pos, m, h, rows=centre)
    rho0 = 0.5 / s ** 3
    assert np.max(np.abs(rho / rho0 - 1.0)) < 0.01
    assert np.all(cnt == cnt[0])
