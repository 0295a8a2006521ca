"""The shared-prefix decomposition of the group walk, restated on the CPU and
checked against the oracle's own interaction lists (no GPU).

The group MAC (a cell is accepted by a group when the nearest point of the
group's particle box lies beyond the cell's opening radius, float32 steps, and
the cell is not an ancestor of the group) has two monotone properties that the
shared walk uses for every group inside an anchor cell A:

* a cell whose opening radius reaches the farthest point of A's box is opened
  by every group inside A (the nearest-point distance of a smaller box, taken
  in the same float32 steps, is never larger);
* a cell that A's box accepts is accepted by every group inside A.

So the lists of a group are exactly A's accepted cells (F) plus what a walk of
the group from the cells A left (S) accepts and opens.  This test builds F and
S in float32 numpy from the oracle's tree and MAC data and compares, for
sampled groups and anchor heights 1 and 3, the union with the oracle's
per-group lists as sets; a dropped or doubled cell, or a wrong decision in
either property, fails it.
"""
import numpy as np
import pytest

from paper_1204_2280_amd import workloads as W

F32 = np.float32


def _near_d2(bmin, bmax, m):
    d = np.maximum(np.maximum(bmin - m, m - bmax), F32(0))
    return F32(F32(d[0] * d[0] + d[1] * d[1]) + d[2] * d[2])


def _far_d2(bmin, bmax, m):
    d = np.maximum(np.maximum(bmax - m, m - bmin), F32(0))
    return F32(F32(d[0] * d[0] + d[1] * d[1]) + d[2] * d[2])


class _Tree:
    def __init__(self, orc, pos, mass, theta):
        self.T = orc.Tree(pos, mass)
        mac = self.T.mac_prep(theta)
        self.com, self.r2 = mac["com32"], mac["r2open"]
        c = self.T.cells()
        self.first, self.count, self.level = c["first"], c["count"], c["level"]
        self.cf, self.nch, self.parent = c["child_first"], c["nchild"], c["parent"]
        mp = self.T.multipoles()
        self.bmin, self.bmax = mp["bmin"], mp["bmax"]
        self.G = self.T.groups()
        self.spos = np.asarray(pos, F32)[self.T.perm]
        self.theta = theta

    def anc(self, c, f0, l0):
        return self.first[c] <= f0 < self.first[c] + self.count[c] and self.level[c] <= l0

    def kids(self, c):
        return list(range(self.cf[c], self.cf[c] + self.nch[c]))

    def anchor_lists(self, A):
        """F (accepted by A's box) and S (left to each group) from the root."""
        bmin, bmax = self.bmin[A], self.bmax[A]
        f0, l0 = self.first[A], self.level[A]
        stack, F, S = [0], [], []
        while stack:
            c = stack.pop()
            m, r2 = self.com[c], self.r2[c]
            if self.anc(c, f0, l0) or not (_far_d2(bmin, bmax, m) > r2):
                if self.nch[c]:
                    stack.extend(self.kids(c))
                else:
                    S.append(c)  # an opened leaf: each group takes it itself
            elif _near_d2(bmin, bmax, m) > r2:
                F.append(c)
            else:
                S.append(c)
        return F, S

    def group_walk(self, g, start):
        """(accepted cells, opened leaves) of group g walking from the cells `start`."""
        f0, n0, l0 = self.G["first"][g], self.G["count"][g], self.G["level"][g]
        p = self.spos[f0:f0 + n0]
        bmin, bmax = p.min(axis=0), p.max(axis=0)
        stack, pc, pp = list(start), [], []
        while stack:
            c = stack.pop()
            if not self.anc(c, f0, l0) and _near_d2(bmin, bmax, self.com[c]) > self.r2[c]:
                pc.append(c)
            elif self.nch[c]:
                stack.extend(self.kids(c))
            else:
                pp.append(c)
        return pc, pp


def _ancestor(t, c, k):
    for _ in range(k):
        if t.level[c] == 0:
            break
        c = t.parent[c]
    return c


@pytest.mark.parametrize("workload", ["plummer", "hernquist"])
def test_anchor_lists_give_the_oracle_lists(orc, workload):
    if workload == "plummer":
        pos, _, mass = W.plummer(20000, 5, with_velocities=False)
    else:
        pos, mass = W.hernquist(12000, 6)
    t = _Tree(orc, pos, mass, 0.75)
    ng = len(t.G["first"])
    sample = np.random.default_rng(0).choice(ng, size=min(60, ng), replace=False)
    shared_total = 0
    for up in (1, 3):
        cache = {}
        for g in sample:
            A = _ancestor(t, t.G["cell"][g], up)
            if A not in cache:
                cache[A] = t.anchor_lists(A)
            F, S = cache[A]
            pc, pp = t.group_walk(g, S)
            pc_o, pp_o = t.T.group_lists(int(g), 0.75)
            assert len(F) + len(pc) == len(pc_o) and not set(F) & set(pc)
            assert set(F) | set(pc) == set(pc_o.tolist())
            assert sorted(pp) == sorted(pp_o.tolist())
            # the plain walk from the root gives the same lists (the restatement itself)
            pc_r, pp_r = t.group_walk(g, [0])
            assert sorted(pc_r) == sorted(pc_o.tolist()) and sorted(pp_r) == sorted(pp_o.tolist())
            shared_total += len(F)
    assert shared_total > 0  # the anchors do decide cells for their groups


def test_rounded_distances_are_monotone_in_the_box():
    """The two facts the anchor lists rest on, in float32 with the kernels'
    operation order: for a box B' inside a box B and any point m, the rounded
    nearest-point squared distance of B' lies between B's nearest-point and
    B's farthest-point squared distances (so B's acceptance implies B''s, and
    a cell B surely opens is opened by B')."""
    rng = np.random.default_rng(11)
    for _ in range(20000):
        scale = F32(10.0) ** F32(rng.integers(-3, 4))
        lo = (rng.standard_normal(3) * scale).astype(F32)
        hi = (lo + np.abs(rng.standard_normal(3)) * scale).astype(F32)
        u, v = np.sort(rng.random((2, 3)), axis=0).astype(F32)
        slo = np.clip((lo + (hi - lo) * u).astype(F32), lo, hi)
        shi = np.clip((lo + (hi - lo) * v).astype(F32), slo, hi)
        m = (rng.standard_normal(3) * scale * F32(3)).astype(F32)
        if rng.random() < 0.5:  # points on box faces and inside, where the clamps matter
            m = np.where(rng.random(3) < 0.5, lo, m).astype(F32)
        near_b, far_b = _near_d2(lo, hi, m), _far_d2(lo, hi, m)
        near_s = _near_d2(slo, shi, m)
        assert near_b <= near_s <= far_b
