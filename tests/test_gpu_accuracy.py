"""Accuracy of the GPU force step against float64 direct summation (the
oracle's direct sum), per opening angle and per accumulation mode.

The paper prints no error figures for its tree-code, so the absolute error
level is not pinned: these tests report it (p50 / p90 / p99 / max of the
relative acceleration and potential errors) and check what the method fixes
regardless of its level: errors fall as theta falls, and Kahan accumulation
changes them by far less than the approximation itself.
  * 2^15 Plummer (seed 1): every particle against the full direct sum.
  * 2^22 Plummer (seed 3): a 4,096-particle subsample (seed 7).
"""
import numpy as np
import pytest

from gpu_helpers import gpu_context, rel_err
from paper_1204_2280_amd import workloads as W

pytestmark = pytest.mark.gpu

THETAS = (0.5, 0.75, 1.0)


def _stats(e):
    return {"p50": float(np.percentile(e, 50)), "p90": float(np.percentile(e, 90)),
            "p99": float(np.sort(e)[int(np.ceil(0.99 * len(e))) - 1]), "max": float(e.max())}


def _errors(orc, n, seed, targets, precisions):
    import torch
    from paper_1204_2280_amd import mibh
    pos, _, mass = W.plummer(n, seed, with_velocities=False)
    ad, pd = orc.direct(pos, mass, targets=targets)
    idx = np.arange(n) if targets is None else targets
    p = torch.from_numpy(pos).cuda()
    m = torch.from_numpy(mass).cuda()
    out = {}
    for prec in precisions:
        ctx = gpu_context(n, precision=prec)
        for theta in THETAS:
            acc, pot = ctx.forces(p, m, theta)
            ctx.sync()
            a = acc.cpu().numpy().astype(np.float64)[idx]
            q = pot.cpu().numpy().astype(np.float64)[idx]
            out[(prec, theta)] = (_stats(rel_err(a, ad)), _stats(rel_err(q, pd)))
            name = "kahan" if prec == mibh.KAHAN else "plain"
            print(f"[gpu] N={n} {name} theta={theta}: acc {out[(prec, theta)][0]} pot {out[(prec, theta)][1]}",
                  flush=True)
        del ctx
    return out


def _check(out, precisions):
    from paper_1204_2280_amd import mibh
    for prec in precisions:
        for k in ("p50", "p90", "p99"):
            e = [out[(prec, t)][0][k] for t in THETAS]
            assert e[0] < e[1] < e[2], (prec, k, e)
    if len(precisions) == 2:
        for t in THETAS:
            pl, ka = out[(mibh.PLAIN, t)][0]["p99"], out[(mibh.KAHAN, t)][0]["p99"]
            assert abs(ka - pl) <= 0.01 * pl


def test_accuracy_vs_direct_summation_2e15(orc):
    from paper_1204_2280_amd import mibh
    precs = (mibh.PLAIN, mibh.KAHAN)
    out = _errors(orc, 1 << 15, 1, None, precs)
    _check(out, precs)
    # the approximation is a few per mille at theta = 0.75 (quadrupole order)
    assert out[(mibh.PLAIN, 0.75)][0]["p50"] < 1e-2


def test_accuracy_vs_direct_summation_2e22_subsample(orc):
    from paper_1204_2280_amd import mibh
    precs = (mibh.PLAIN, mibh.KAHAN)
    out = _errors(orc, 1 << 22, 3, W.subsample(1 << 22, 4096, 7), precs)
    _check(out, precs)
    assert out[(mibh.PLAIN, 0.75)][0]["p50"] < 1e-2
