"""The autotuner times every candidate, respects the accuracy limit, and caches."""
import json

import numpy as np
import pytest

from paper_1204_2280_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_autotune_small_grid(tmp_path, monkeypatch):
    import torch
    from paper_1204_2280_amd import autotune
    monkeypatch.setenv("MIBH_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    pos, mass, off = W.ensemble(4, 11, 10, 13)
    dev = torch.device("cuda", 0)
    p = torch.from_numpy(pos).to(dev)
    m = torch.from_numpy(mass).to(dev)
    grid = {"ncrit": (8, 16), "group_cap": (32, 64), "walk_waves": (1024,)}
    best, cands = autotune.tune(p, m, off, 0.75, grid=grid, steps=2, max_rel_diff=1e-2)
    assert len(cands) == 4
    assert all(c["ms_per_step"] > 0 for c in cands)
    ok = [c for c in cands if c["p99_rel_diff_vs_default"] <= 1e-2]
    assert best == {k: min(ok, key=lambda c: c["ms_per_step"])[k] for k in ("ncrit", "group_cap", "walk_waves")}
    cached = json.load(open(tmp_path / "tune.json"))
    assert len(cached) == 1
    best2, _ = autotune.tune(p, m, off, 0.75, grid=grid)
    assert best2 == best
