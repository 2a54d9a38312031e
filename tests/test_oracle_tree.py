"""Pins for the oracle's octree and interaction lists (section "Computational
structure of FMM operators": n_crit, the U/V/W/X lists, their bounds under
the 2:1 balance condition)."""
import numpy as np
import pytest

from oracle.octree import Octree
from paper_2303_08394_amd import inputs as I


def _uniform_pair_counts(depth):
    """Exact U and V pair totals of a full uniform grid, from 1-D counts.

    V(B) = (children of parent's colleagues) minus (adjacent boxes): both sets
    are boxes of per-axis index ranges, so totals factorise over the axes."""
    u_tot = None
    v_tot = 0
    for level in range(2, depth + 1):
        n = 2 ** level
        a = 0  # sum over i of #children of parent colleagues (1-D)
        b = 0  # sum over i of #adjacent indices (1-D)
        for i in range(n):
            p = i // 2
            parents = [j for j in (p - 1, p, p + 1) if 0 <= j < n // 2]
            a += 2 * len(parents)
            b += len([j for j in (i - 1, i, i + 1) if 0 <= j < n])
        v_tot += a ** 3 - b ** 3
        u_tot = b ** 3
    return u_tot, v_tot


def test_uniform_counts_closed_form():
    # exact grid counts: depth 3 -> 10,648 U and 56,448 V pairs
    assert _uniform_pair_counts(3) == (10648, 56448)
    assert _uniform_pair_counts(5) == (830584, 6039504)
    x, _ = I.uniform_cube(20000, seed=0)
    t = Octree(x, x, uniform_depth=3, center=(0.5, 0.5, 0.5), halfwidth=0.5)
    leaves = t.leaves()
    assert len(leaves) == 512 and all(t.level[b] == 3 for b in leaves)
    nu = sum(len(t.U(b)) for b in leaves)
    nv = sum(len(t.V(b)) for b in range(len(t.level)))
    assert (nu, nv) == _uniform_pair_counts(3)
    assert max(len(t.V(b)) for b in range(len(t.level))) == 189
    assert all(len(t.W(b)) == 0 and len(t.X(b)) == 0 for b in leaves)


def _partition_ok(t, pts, ids_attr):
    seen = np.zeros(len(pts), dtype=int)
    for b in t.leaves():
        ids = getattr(t, ids_attr)[b]
        seen[ids] += 1
        c, r = t.center(b), t.halfwidth(t.level[b])
        assert np.all(np.abs(pts[ids] - c) <= r * (1 + 1e-12))
    assert np.all(seen == 1)


def _descendant_or_self(t, a, s):
    while s >= 0:
        if s == a:
            return True
        s = t.parent[s]
    return False


def _coverage_ok(t):
    """Every (target leaf, source leaf) pair is covered exactly once by
    U(B), W(B), or V/X of B or one of its ancestors."""
    leaves = t.leaves()
    for b in leaves:
        chain = []
        a = b
        while a >= 0:
            chain.append(a)
            a = t.parent[a]
        for s in leaves:
            cnt = int(s in t.U(b))
            cnt += sum(_descendant_or_self(t, a, s) for a in t.W(b))
            for c in chain:
                cnt += sum(_descendant_or_self(t, a, s) for a in t.V(c))
                cnt += sum(a == s for a in t.X(c))
            assert cnt == 1, (b, s, cnt)


def _balanced(t):
    leaves = t.leaves()
    for i, a in enumerate(leaves):
        for b in leaves[i + 1:]:
            if abs(t.level[a] - t.level[b]) > 1 and t.adjacent(a, b):
                return False
    return True


def test_uniform_coverage_and_partition():
    x, _ = I.uniform_cube(3000, seed=3)
    t = Octree(x, x, uniform_depth=2, center=(0.5, 0.5, 0.5), halfwidth=0.5)
    _partition_ok(t, x, "srcs")
    _coverage_ok(t)


@pytest.mark.parametrize("kind", ["sphere", "clustered"])
def test_adaptive_tree_properties(kind):
    if kind == "sphere":
        x, _ = I.sphere_surface(4000, seed=0)
        t = Octree(x, x, ncrit=24, max_depth=8)
    else:
        x, _ = I.clustered(4000, seed=5, sigma=0.05)
        t = Octree(x, x, ncrit=24, max_depth=8, center=(0.5, 0.5, 0.5), halfwidth=0.5)
    _partition_ok(t, x, "srcs")
    _partition_ok(t, x, "tgts")
    assert _balanced(t)
    leaves = t.leaves()
    assert len(set(t.level[b] for b in leaves)) >= 2
    for b in leaves:
        assert len(t.srcs[b]) <= 24 or t.level[b] == 8
        assert len(t.U(b)) <= 60 and len(t.W(b)) <= 152
    nb = len(t.level)
    assert max(len(t.V(b)) for b in range(nb)) <= 189
    assert max(len(t.X(b)) for b in range(nb)) <= 19
    # the adaptive lists are really exercised
    assert sum(len(t.W(b)) for b in leaves) > 0
    assert sum(len(t.X(b)) for b in range(nb)) > 0
    # X is the transpose of W
    wpairs = {(a, b) for b in leaves for a in t.W(b)}
    xpairs = {(b, a) for b in range(nb) for a in t.X(b)}
    assert wpairs == xpairs


def test_adaptive_coverage_small():
    x, _ = I.clustered(1500, seed=7, sigma=0.06)
    t = Octree(x, x, ncrit=16, max_depth=7, center=(0.5, 0.5, 0.5), halfwidth=0.5)
    assert len(set(t.level[b] for b in t.leaves())) >= 3
    _coverage_ok(t)


def test_separate_targets_and_unbalanced():
    rng = np.random.default_rng(9)
    src = I.clustered(800, seed=9)[0]
    tgt = rng.random((500, 3))
    t = Octree(src, tgt, ncrit=10, max_depth=7, balance=False,
               center=(0.5, 0.5, 0.5), halfwidth=0.5)
    _partition_ok(t, src, "srcs")
    _partition_ok(t, tgt, "tgts")
    _coverage_ok(t)


def test_root_from_data_and_boundary_rule():
    x = np.array([[0.0, 0.0, 0.0], [1.0, 2.0, 0.5], [0.5, 1.0, 0.25]])
    t = Octree(x, x, uniform_depth=1)
    np.testing.assert_allclose(t.c0, [0.5, 1.0, 0.25])
    assert t.r0 == pytest.approx(1.0 * (1 + 2 ** -20), rel=1e-15)
    # the centre point lies on the internal faces: it goes to the upper box
    assert tuple(Octree.point_index(t.ts[2:3], 1)[0]) == (1, 1, 1)
    # points on the root's upper face are clamped into the last box
    assert np.all(Octree.point_index(np.array([[1.0, 1.0, 1.0]]), 3) == 7)
