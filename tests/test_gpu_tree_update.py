"""Device re-sort of a tree's points (kifmm_tree_update_points) against the
host build on the same points and the FP64 oracle.

Bit-exact where the work is integer or follows the host's FP64 rules: the
sorted order, every box's point ranges, and the evaluation (equal inputs in
equal order give equal potentials, bitwise).  The potentials of the updated
tree also meet the oracle at the mixed-precision tolerance.  Cases cover two
to eight radix passes (uniform depths 3, 5, 6; adaptive trees keyed at
levels 10, 16 and 20), a resident forest updated in place (also under graph
replay) and one refreshed through the host copy, separate targets, and the
rejected cases.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import kifmm as OK  # noqa: E402
from oracle.octree import Octree  # noqa: E402
from paper_2303_08394_amd import inputs as I  # noqa: E402
from paper_2303_08394_amd import kifmm as K  # noqa: E402

DEV = "cuda:0"
CUBE = dict(center=(0.5, 0.5, 0.5), halfwidth=0.5)
_ops = {}


def ops(p):
    if p not in _ops:
        _ops[p] = K.Operators(p)
    return _ops[p]


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def evaluate(tree, q, p, precision="fp32"):
    out = K.evaluate(tree, ops(p), dev(np.atleast_2d(q)), precision=precision)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def same_leaves(x, depth, seed):
    """New points, each in the leaf cell of the old one (fresh position inside
    it): the occupied leaves stay the same, the order inside them changes."""
    cells = 2 ** depth
    c = np.clip(np.floor(x * cells), 0, cells - 1)
    u = np.random.default_rng(seed).random(x.shape)
    return (c + u) / cells


def assert_same_tree(a, b):
    ba, bb = a.boxes(), b.boxes()
    for k in ("level", "anchor", "is_leaf", "src_range", "tgt_range"):
        np.testing.assert_array_equal(ba[k], bb[k])
    for pa, pb in zip(a.perm(), b.perm()):
        np.testing.assert_array_equal(pa, pb)


@pytest.mark.parametrize("n,depth", [(20000, 3), (60000, 5), (150000, 6)])
@pytest.mark.parametrize("evaluated_first", [True, False])
def test_update_equals_host_build(n, depth, evaluated_first):
    x0, q = I.uniform_cube(n, seed=40 + depth)
    x1 = same_leaves(x0, depth, seed=50 + depth) if depth >= 5 else I.uniform_cube(n, seed=60)[0]
    p = 4
    tree = K.Tree(x0, uniform_depth=depth, **CUBE)
    if evaluated_first:
        evaluate(tree, q, p)  # a forest resident on the device takes the update in place
    tree.update_points(dev(x1))
    torch.cuda.synchronize()
    fresh = K.Tree(x1, uniform_depth=depth, **CUBE)
    got = evaluate(tree, q, p)
    want = evaluate(fresh, q, p)
    np.testing.assert_array_equal(got, want)
    assert_same_tree(tree, fresh)


def test_update_matches_oracle_and_graph_replays():
    """Updated points seen by a captured graph: replays after the update give
    the new tree's potentials (bitwise those of a fresh tree), which meet the
    oracle."""
    n, depth, p = 12000, 3, 5
    x0, q = I.uniform_cube(n, seed=70, charge_range=(-1, 1))
    x1 = I.uniform_cube(n, seed=71)[0]
    tree = K.Tree(x0, uniform_depth=depth, **CUBE)
    qd = dev(q)
    out = torch.empty((1, n), dtype=torch.float64, device=DEV)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        K.evaluate(tree, ops(p), qd, precision="bf16x3", out=out)  # captured
        K.evaluate(tree, ops(p), qd, precision="bf16x3", out=out)  # replayed
        tree.update_points(dev(x1), stream=s)
        K.evaluate(tree, ops(p), qd, precision="bf16x3", out=out)  # replayed on the new order
        torch.cuda.synchronize()
        got = out.cpu().numpy()
    fresh = K.Tree(x1, uniform_depth=depth, **CUBE)
    want_gpu = evaluate(fresh, q, p, "bf16x3")
    np.testing.assert_array_equal(got, want_gpu)
    want = OK.KIFMM(Octree(x1, x1, uniform_depth=depth, **CUBE), p).evaluate(np.atleast_2d(q))
    assert rel(got, want) < 1e-5


def test_update_separate_targets():
    n, m, depth, p = 15000, 9000, 3, 4
    xs0, q = I.uniform_cube(n, seed=80)
    xt0 = I.uniform_cube(m, seed=81)[0]
    xs1, xt1 = I.uniform_cube(n, seed=82)[0], I.uniform_cube(m, seed=83)[0]
    tree = K.Tree(xs0, xt0, uniform_depth=depth, **CUBE)
    evaluate(tree, q, p)
    with pytest.raises(K.KifmmError, match="targets"):
        tree.update_points(dev(xs1))
    tree.update_points(dev(xs1), dev(xt1))
    fresh = K.Tree(xs1, xt1, uniform_depth=depth, **CUBE)
    np.testing.assert_array_equal(evaluate(tree, q, p), evaluate(fresh, q, p))
    assert_same_tree(tree, fresh)


def test_update_rejects_other_leaves_and_keeps_tree():
    n, depth, p = 20000, 3, 4
    x0, q = I.uniform_cube(n, seed=90)
    tree = K.Tree(x0, uniform_depth=depth, **CUBE)
    before = evaluate(tree, q, p)
    squeezed = 0.5 * x0  # every point in the lower octant: other leaves empty
    with pytest.raises(K.KifmmError, match="leaves"):
        tree.update_points(dev(squeezed))
    np.testing.assert_array_equal(evaluate(tree, q, p), before)
    L = K.lib()
    assert L.kifmm_tree_update_points(tree.handle, None, None, None) == 1  # EINVAL: null
    with pytest.raises(K.KifmmError, match="device memory"):  # host memory is refused
        K._check(L.kifmm_tree_update_points(tree.handle, K._dptr(x0), None, None))
    np.testing.assert_array_equal(evaluate(tree, q, p), before)


def test_update_rejects_points_outside_the_root_and_keeps_tree():
    """A point moved past the root cube would be clamped into a boundary
    leaf, outside that leaf's equivalent surface: the update is refused and
    the tree evaluates as before."""
    n, depth, p = 20000, 3, 4
    x0, q = I.uniform_cube(n, seed=91)
    tree = K.Tree(x0, uniform_depth=depth, **CUBE)
    before = evaluate(tree, q, p)
    for bad_value in (1.0 + 1e-9, -1e-12):
        moved = x0.copy()
        moved[123, 1] = bad_value
        with pytest.raises(K.KifmmError, match="outside the tree's root box"):
            tree.update_points(dev(moved))
        np.testing.assert_array_equal(evaluate(tree, q, p), before)
    # the auto root (bounding cube with a 2^-20 margin) of an adaptive tree
    tree2 = K.Tree(x0, ncrit=64, max_depth=8)
    inf = tree2.info()
    moved = x0.copy()
    moved[7, 0] = inf.root_center[0] + 1.01 * inf.root_halfwidth
    with pytest.raises(K.KifmmError, match="outside the tree's root box"):
        tree2.update_points(dev(moved))


def test_update_fullsize_1m():
    """1M points, depth 5: the device sort agrees with the host build."""
    prob = I.uniform_1m()
    x1 = I.uniform_cube(prob.n, seed=123)[0]
    tree = K.Tree(prob.points, uniform_depth=prob.uniform_depth, center=prob.center, halfwidth=prob.halfwidth)
    evaluate(tree, prob.charges[0], prob.p)
    tree.update_points(dev(x1))
    fresh = K.Tree(x1, uniform_depth=prob.uniform_depth, center=prob.center, halfwidth=prob.halfwidth)
    assert_same_tree(tree, fresh)


def inside_own_leaves(tree, seed):
    """New caller-order points, each drawn inside the leaf cube that holds the
    old one: every leaf keeps its points (and its count)."""
    bx, inf = tree.boxes(), tree.info()
    sperm, _ = tree.perm()
    lo = np.asarray(inf.root_center) - inf.root_halfwidth
    n = inf.n_src
    new = np.empty((n, 3))
    u = np.random.default_rng(seed).random((n, 3))
    for b in np.nonzero(bx["is_leaf"] == 1)[0]:
        s0, s1 = bx["src_range"][b]
        if s1 <= s0:
            continue
        w = 2 * inf.root_halfwidth / 2 ** int(bx["level"][b])
        idx = sperm[s0:s1]
        new[idx] = lo + (bx["anchor"][b] + u[idx]) * w
    return new


@pytest.mark.parametrize("max_depth,ncrit", [(10, 32), (16, 24), (20, 24)])
def test_update_adaptive_equals_host_build(max_depth, ncrit):
    x0, q = I.sphere_surface(20000, seed=100 + max_depth, jitter=0.0)
    p = 4
    tree = K.Tree(x0, ncrit=ncrit, max_depth=max_depth)
    inf = tree.info()
    evaluate(tree, q, p)
    x1 = inside_own_leaves(tree, seed=7)
    tree.update_points(dev(x1))
    fresh = K.Tree(x1, ncrit=ncrit, max_depth=max_depth, center=tuple(inf.root_center),
                   halfwidth=inf.root_halfwidth)
    assert fresh.info().n_boxes == inf.n_boxes
    assert_same_tree(tree, fresh)
    np.testing.assert_array_equal(evaluate(tree, q, p), evaluate(fresh, q, p))


def test_repeated_updates_then_host_export():
    """Several updates in a row on an evaluated tree (the forest takes each in
    place), then the host copy (exports, a plan rebuild) reflects the last."""
    n, depth, p = 30000, 4, 4
    x0, q = I.uniform_cube(n, seed=130)
    tree = K.Tree(x0, uniform_depth=depth, **CUBE)
    evaluate(tree, q, p)
    xs = [same_leaves(x0, depth, seed=131 + k) for k in range(3)]
    for x in xs:
        tree.update_points(dev(x))
        got = evaluate(tree, q, p)
    fresh = K.Tree(xs[-1], uniform_depth=depth, **CUBE)
    np.testing.assert_array_equal(got, evaluate(fresh, q, p))
    assert_same_tree(tree, fresh)
    K.set_tuning("m2l_tile_cols", 128)  # new plans: built from the refreshed host copy
    try:
        np.testing.assert_array_equal(evaluate(tree, q, p), evaluate(fresh, q, p))
    finally:
        K.set_tuning("m2l_tile_cols", 64)
