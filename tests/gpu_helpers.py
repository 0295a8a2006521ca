"""Shared helpers for the GPU parity tests (runs the HIP path and the oracle)."""
from __future__ import annotations

import numpy as np

# float32 interactions vs the float64 oracle: relative error of each particle's
# acceleration (and potential), 99th percentile (nearest rank)
TOL_P99 = 1e-5


def gpu_context(n_max, **params):
    import torch
    from paper_1204_2280_amd import mibh
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    mibh.lib()  # raises if the HIP library was not built
    return mibh.Context(n_max, **params)


def run_gpu(ctx, pos, mass, theta, exports=("keys", "perm", "cells", "groups", "counts", "multipoles",
                                            "delta", "mac", "spos")):
    import torch
    p = torch.from_numpy(np.ascontiguousarray(pos, np.float32)).to(ctx.device)
    m = torch.from_numpy(np.ascontiguousarray(mass, np.float32)).to(ctx.device)
    acc, pot = ctx.forces(p, m, theta)
    ctx.sync()
    out = {"acc": acc.cpu().numpy().astype(np.float64), "pot": pot.cpu().numpy().astype(np.float64)}
    from paper_1204_2280_amd.mibh import Decoded
    for e in exports:
        t = ctx.export(e)
        if e == "cells":
            out[e] = Decoded.cells(t)
        elif e == "groups":
            out[e] = Decoded.groups(t)
        elif e == "keys":
            out[e] = t.cpu().numpy().view(np.uint64)
        elif e in ("perm",):
            out[e] = t.cpu().numpy().view(np.uint32).astype(np.int64)
        elif e == "counts":
            out[e] = t.cpu().numpy().view(np.uint32).astype(np.int64)
        else:
            out[e] = t.cpu().numpy()
    return out


def rel_err(a, ref):
    a = np.asarray(a, np.float64)
    ref = np.asarray(ref, np.float64)
    if a.ndim == 2:
        num = np.linalg.norm(a - ref, axis=1)
        den = np.linalg.norm(ref, axis=1)
    else:
        num = np.abs(a - ref)
        den = np.abs(ref)
    return num / np.where(den > 0, den, 1.0)


def term_scale(pos, mass, G=1.0):
    """S_i = sum_j G m_j / r_ij^2: the summed magnitude of particle i's direct
    terms.  float32 evaluation of a sum with condition S_i/|a_i| can only be
    expected to reach |error| ~ u * S_i, so ill-conditioned edge cases (points
    on a line, coincident clumps) are checked with |error| / S_i."""
    x = np.asarray(pos, np.float64)
    m = np.asarray(mass, np.float64)
    S = np.zeros(len(m))
    for b in range(0, len(m), 512):
        d = x[None, :, :] - x[b:b + 512, None, :]
        r2 = np.sum(d * d, axis=2)
        with np.errstate(divide="ignore"):
            w = np.where(r2 > 0, m[None, :] / r2, 0.0)
        S[b:b + 512] = G * w.sum(axis=1)
    return S


def p99(e):
    e = np.sort(np.asarray(e))
    if e.size == 0:
        return 0.0
    return float(e[int(np.ceil(0.99 * e.size)) - 1])


def assert_tree_equal(g, T):
    """Keys, permutation, moved particles, cells and groups bit for bit."""
    np.testing.assert_array_equal(g["keys"], T.keys)
    np.testing.assert_array_equal(g["perm"], T.perm)
    oc = T.cells()
    for f in ("first", "count", "child_first", "level", "nchild"):
        np.testing.assert_array_equal(g["cells"][f], oc[f], err_msg=f"cells.{f}")
    og = T.groups()
    for f in ("first", "count", "level"):
        np.testing.assert_array_equal(g["groups"][f], og[f], err_msg=f"groups.{f}")


def assert_multipoles_equal(g, T, theta):
    mp = T.multipoles()
    gm = g["multipoles"]
    np.testing.assert_array_equal(gm[:, 0], mp["M"])
    np.testing.assert_array_equal(gm[:, 1:4], mp["com"])
    np.testing.assert_array_equal(gm[:, 4:10], mp["S"])
    np.testing.assert_array_equal(g["delta"], mp["delta"])
    mac = T.mac_prep(theta)
    np.testing.assert_array_equal(g["mac"][:, :3], mac["com32"])
    np.testing.assert_array_equal(g["mac"][:, 3], mac["r2open"])
