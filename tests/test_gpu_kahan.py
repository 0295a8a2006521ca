"""Accumulation modes of the walk against the float64 oracle on the same
interaction lists: plain float32 (MIBH_PLAIN), Kahan compensation of the
totals of successive list evaluations (MIBH_KAHAN) and of every term
(MIBH_KAHAN_TERM).

Within one evaluation a lane sums at most 16 tiles and the lanes are folded
by a six-level tree, so a particle's plain float32 sum is long only across
evaluations (one per flush of a full list).  Where lists are short (Plummer
at theta = 0.75, two or three evaluations per group) the three modes agree to
rounding noise; where they are long (theta = 1e-4 opens every cell: each
group evaluates all 2^15 particles in 64 flushes of its 512-entry list) the
compensated modes must cut the error.  The line and the coincident clump
(net forces a tiny fraction of their terms) are dominated by the error of
the terms themselves, which no compensation of the sum removes: there the
modes must agree within a few per cent of each other.  Counts are identical
in every mode.
"""
import numpy as np
import pytest

from gpu_helpers import TOL_P99, gpu_context, p99, rel_err, run_gpu
from paper_1204_2280_amd import workloads as W

pytestmark = pytest.mark.gpu

MODES = ((0, "plain"), (1, "kahan"), (2, "kahan_term"))


def _inputs(name):
    if name == "plummer_32k":
        p, _, m = W.plummer(32768, 1, with_velocities=False)
    elif name == "line_2000":
        p = np.zeros((2000, 3), np.float32)
        p[:, 1] = np.linspace(-3, 5, 2000, dtype=np.float32)
        m = np.full(2000, 1 / 2000, np.float32)
    elif name == "coincident_300":
        p = np.tile(np.array([[0.25, -0.5, 0.125]], np.float32), (300, 1))
        p = np.concatenate([p, W.uniform_cube(50, 3)[0]])
        m = np.full(350, 1 / 350, np.float32)
    else:
        raise KeyError(name)
    return np.ascontiguousarray(p, np.float32), np.ascontiguousarray(m, np.float32)


def _errors(orc, name, theta):
    pos, mass = _inputs(name)
    T = orc.Tree(pos, mass)
    T.walk(theta)
    acc, pot = T.forces()
    npc, npp = T.counts()
    out = {}
    for prec, label in MODES:
        c = gpu_context(len(mass), precision=prec)
        g = run_gpu(c, pos, mass, theta, exports=("counts",))
        np.testing.assert_array_equal(g["counts"][:, 0], npc)
        np.testing.assert_array_equal(g["counts"][:, 1], npp)
        e = rel_err(g["acc"], acc)
        ep = rel_err(g["pot"], pot)
        out[label] = {"p50": float(np.median(e)), "p99": p99(e), "rms": float(np.sqrt(np.mean(e ** 2))),
                      "pot_p99": p99(ep)}
        print(f"[gpu] accumulation {name} theta={theta} {label}: {out[label]}", flush=True)
    return out


def test_short_lists_modes_agree(orc):
    out = _errors(orc, "plummer_32k", 0.75)
    for label in ("plain", "kahan", "kahan_term"):
        assert out[label]["p99"] <= TOL_P99 and out[label]["pot_p99"] <= TOL_P99
    # rounding noise only: within 5% of each other at p99 and in RMS
    for label in ("kahan", "kahan_term"):
        assert out[label]["p99"] <= 1.05 * out["plain"]["p99"]
        assert out[label]["rms"] <= 1.05 * out["plain"]["rms"]


def test_long_lists_compensation_cuts_the_error(orc):
    out = _errors(orc, "plummer_32k", 1e-4)
    for label in ("kahan", "kahan_term"):
        assert out[label]["p50"] < 0.8 * out["plain"]["p50"], out
        assert out[label]["rms"] < 0.8 * out["plain"]["rms"], out
        assert out[label]["p99"] <= out["plain"]["p99"], out


@pytest.mark.parametrize("name", ["line_2000", "coincident_300"])
def test_ill_conditioned_term_error_dominates(orc, name):
    out = _errors(orc, name, 0.75)
    for label in ("kahan", "kahan_term"):
        assert out[label]["p99"] <= 1.05 * out["plain"]["p99"], out
