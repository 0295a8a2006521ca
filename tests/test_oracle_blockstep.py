"""Pins of the oracle's block time steps.

* One level and a rebuild every tick is the shared-step leapfrog, bit for bit.
* A light particle on an eccentric orbit about a heavy one (pericentre 0.2,
  apocentre 1.8): the block scheme spends its small steps near pericentre; its
  energy error is far below that of shared steps of dt_max and within a
  small factor of shared steps of dt_max / 2^R, with far fewer force
  evaluations than the latter.
* Step levels follow the criterion: 16^r >= dt_max^4 |a|^2 / (eta^4 eps^2).
"""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def bs(orc):
    from oracle import blockstep
    return blockstep


def _kepler():
    # heavy mass 1 at the origin, light mass 1e-6 at apocentre 1.8 moving slowly
    ra, rp = 1.8, 0.2
    a_orb = 0.5 * (ra + rp)
    va = np.sqrt((2.0 / ra - 1.0 / a_orb))  # vis-viva, GM = 1
    x = np.array([[0.0, 0.0, 0.0], [ra, 0.0, 0.0]], np.float32)
    v = np.array([[0.0, 0.0, 0.0], [0.0, va, 0.0]], np.float32)
    m = np.array([1.0, 1e-6], np.float32)
    period = 2 * np.pi * np.sqrt(a_orb ** 3)
    return x, v, m, period


def test_one_level_rebuilding_every_tick_is_the_leapfrog(bs):
    from oracle import leapfrog as lf
    from paper_1204_2280_amd import workloads as W
    pos, vel, mass = W.plummer(500, 17)
    x1, v1, a1, p1, lev, st, log = bs.block_run(pos, vel, mass, 0.75, 1 / 64, 0, 0.1, 0.01, 6, tol=-1.0)
    x2, v2, a2, p2, log2 = lf.leapfrog(pos, vel, mass, 0.75, 1 / 64, 6, log_every=1)
    np.testing.assert_array_equal(x1, x2)
    np.testing.assert_array_equal(v1, v2)
    np.testing.assert_array_equal(log, log2)
    assert st["rebuilds"] == 6 and st["substeps"] == 6 and np.all(lev == 0)


def test_eccentric_orbit_block_steps(bs):
    from oracle import leapfrog as lf
    x, v, m, period = _kepler()
    R = 6
    nbig = 16
    dt_max = period / nbig
    xb, vb, _, _, lev, st, log = bs.block_run(x, v, m, 0.75, dt_max, R, 0.05, 1.0, nbig, tol=-1.0)
    Eb = log[:, 1] + log[:, 2]
    err_block = np.abs(Eb - Eb[0]).max() / abs(Eb[0])
    _, _, _, _, lb = lf.leapfrog(x, v, m, 0.75, dt_max, nbig, log_every=1)
    Eb2 = lb[:, 1] + lb[:, 2]
    err_big = np.abs(Eb2 - Eb2[0]).max() / abs(Eb2[0])
    nsmall = nbig << R
    _, _, _, _, ls = lf.leapfrog(x, v, m, 0.75, dt_max / (1 << R), nsmall, log_every=1 << R)
    Es = ls[:, 1] + ls[:, 2]
    err_small = np.abs(Es - Es[0]).max() / abs(Es[0])
    light_updates = st["active_updates"] - st["substeps"] // (1 << R)  # the heavy one stays at level 0
    print(f"energy error: block {err_block:.3e}, shared dt_max {err_big:.3e}, shared dt_min {err_small:.3e}; "
          f"light-particle updates {light_updates} of {nsmall}")
    assert err_block < 0.05 * err_big
    assert err_block < 20 * err_small
    # the light particle is due on far fewer ticks than every tick
    assert light_updates < 0.6 * nsmall


def test_levels_follow_the_criterion(bs):
    rng = np.random.default_rng(2)
    a = rng.standard_normal((1000, 3)) * 10.0 ** rng.uniform(-3, 3, (1000, 1))
    dt_max, eta, eps, R = 0.125, 0.2, 0.01, 8
    r = bs.level_of(a, dt_max, eta, eps, R)
    amag = np.linalg.norm(a, axis=1)
    dt = eta * np.sqrt(eps / amag)
    for i in range(len(r)):
        if r[i] < R:  # dt_max / 2^r <= dt < dt_max / 2^(r-1)
            assert dt_max / 2 ** r[i] <= dt[i] * (1 + 1e-12)
        if r[i] > 0:
            assert dt_max / 2 ** (r[i] - 1) > dt[i] * (1 - 1e-12)
    assert r.min() == 0 and r.max() == R
