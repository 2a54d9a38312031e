"""Host-side checks of the C ABI (no GPU): symbols, error paths, the C++ tree
and lists against the oracle's independent tree, and the FP64 precompute."""
import os
import re

import numpy as np
import pytest

from oracle import kifmm as OK
from oracle.direct import kernel_matrix
from oracle.octree import Octree
from oracle.surface import surface_grid
from paper_2303_08394_amd import inputs as I
from paper_2303_08394_amd import kifmm as K

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CUBE = dict(center=(0.5, 0.5, 0.5), halfwidth=0.5)


def test_every_declared_symbol_is_exported():
    hdr = open(os.path.join(ROOT, "include", "kifmm.h")).read()
    declared = set(re.findall(r"\b(kifmm_\w+)\s*\(", hdr))
    assert len(declared) >= 18
    L = K.lib()
    for name in declared:
        assert hasattr(L, name), name
    assert declared == set(K.EXPORTED)


def _tree_pair(x, tgt=None, **kw):
    tgt = x if tgt is None else tgt
    ot = Octree(x, tgt, **kw)
    ct = K.Tree(x, tgt, **kw)
    return ot, ct


def _compare_trees(ot, ct):
    cb = ct.boxes()
    inf = ct.info()
    assert inf.n_boxes == len(ot.level)
    np.testing.assert_allclose(inf.root_center[:], ot.c0, rtol=0, atol=0)
    assert inf.root_halfwidth == ot.r0
    key = {(int(cb["level"][b]),) + tuple(int(v) for v in cb["anchor"][b]): b for b in range(inf.n_boxes)}
    o2c = {}
    sperm, tperm = ct.perm()
    for ob in range(len(ot.level)):
        k = (ot.level[ob],) + ot.anchor[ob]
        assert k in key, k
        cbx = key[k]
        o2c[ob] = cbx
        assert bool(cb["is_leaf"][cbx]) == ot.is_leaf(ob)
        s0, s1 = cb["src_range"][cbx]
        t0, t1 = cb["tgt_range"][cbx]
        assert sorted(sperm[s0:s1].tolist()) == sorted(ot.srcs[ob].tolist())
        assert sorted(tperm[t0:t1].tolist()) == sorted(ot.tgts[ob].tolist())
    nsrc = {b: len(ot.srcs[b]) for b in range(len(ot.level))}
    for which, fn in ((K.LIST_U, ot.U), (K.LIST_V, ot.V), (K.LIST_W, ot.W), (K.LIST_X, ot.X)):
        off, items = ct.list(which)
        for ob in range(len(ot.level)):
            if len(ot.tgts[ob]) == 0:
                continue
            want = sorted(o2c[a] for a in fn(ob) if nsrc[a] > 0)
            c = o2c[ob]
            got = sorted(items[off[c]:off[c + 1]].tolist())
            assert got == want, (which, ob)
    return o2c


def test_uniform_tree_matches_oracle():
    x, _ = I.uniform_cube(5000, seed=1)
    ot, ct = _tree_pair(x, uniform_depth=3, **CUBE)
    _compare_trees(ot, ct)
    assert ct.info().n_v == 56448 and ct.info().n_u == 10648


@pytest.mark.parametrize("case", ["sphere", "clustered", "separate", "unbalanced", "root_from_data"])
def test_adaptive_tree_matches_oracle(case):
    if case == "sphere":
        x, _ = I.sphere_surface(6000, seed=2)
        ot, ct = _tree_pair(x, ncrit=20, max_depth=9)
    elif case == "clustered":
        x, _ = I.clustered(6000, seed=3)
        ot, ct = _tree_pair(x, ncrit=24, max_depth=9, **CUBE)
    elif case == "separate":
        x, _ = I.clustered(3000, seed=4)
        t = np.random.default_rng(4).random((2000, 3))
        ot, ct = _tree_pair(x, t, ncrit=16, max_depth=8, **CUBE)
    elif case == "unbalanced":
        x, _ = I.clustered(3000, seed=5, sigma=0.03)
        ot, ct = _tree_pair(x, ncrit=16, max_depth=9, balance=False, **CUBE)
    else:
        x, _ = I.sphere_surface(3000, seed=6)
        ot, ct = _tree_pair(x + 3.0, ncrit=30, max_depth=8)
    _compare_trees(ot, ct)
    inf = ct.info()
    if case != "unbalanced":
        assert inf.n_w > 0 and inf.n_x > 0


def test_points_on_faces_and_duplicates():
    # points exactly on internal faces, on the root's upper face, and repeated
    g = np.array([0.0, 0.25, 0.5, 0.75, 1.0])
    x = np.array([(a, b, c) for a in g for b in g for c in g])
    x = np.vstack([x, x[:10]])
    ot, ct = _tree_pair(x, ncrit=4, max_depth=5, **CUBE)
    _compare_trees(ot, ct)


def test_points_outside_a_given_root_are_refused():
    """With a given root box a point outside the closed cube would be clamped
    into a boundary leaf (beyond its equivalent surface): refused.  Points on
    the closed faces are inside."""
    x = np.random.default_rng(3).random((100, 3))
    for bad in (1.0 + 1e-12, -1e-15, 2.0):
        y = x.copy()
        y[17, 2] = bad
        with pytest.raises(K.KifmmError, match="outside the given root box"):
            K.Tree(y, uniform_depth=2, **CUBE)
        with pytest.raises(K.KifmmError, match="outside the given root box"):
            K.Tree(x, y, ncrit=8, max_depth=6, **CUBE)
    y = x.copy()
    y[0] = (0.0, 1.0, 1.0)
    assert K.Tree(y, uniform_depth=2, **CUBE).info().n_src == 100
    # the derived root always holds every point
    assert K.Tree(3.0 * y - 7.0, ncrit=8, max_depth=6).info().n_src == 100


def test_jacobi_svd_pinv_matches_library():
    s = surface_grid(6)
    for p in (2, 4, 6):
        ops = K.Operators(p)
        s = surface_grid(p)
        ref_u = OK.pinv_truncated(kernel_matrix(2.95 * s, 1.05 * s), 1e-9)
        ref_d = OK.pinv_truncated(kernel_matrix(1.05 * s, 2.95 * s), 1e-9)
        # conditioning 1e9 at p=6 makes two correct pinvs differ by ~1e-8
        tol = {2: 1e-13, 4: 1e-10, 6: 1e-7}[p]
        assert np.linalg.norm(ops.export(1) - ref_u) / np.linalg.norm(ref_u) < tol
        assert np.linalg.norm(ops.export(2) - ref_d) / np.linalg.norm(ref_d) < tol
        np.testing.assert_allclose(ops.export(0), s, rtol=0, atol=1e-15)


def test_translation_tables_match_oracle():
    ops = K.Operators(4)
    one = Octree(np.zeros((1, 3)), np.zeros((1, 3)), uniform_depth=0, center=(0, 0, 0), halfwidth=1.0)
    two = Octree(np.zeros((1, 3)), np.zeros((1, 3)), uniform_depth=0, center=(0, 0, 0), halfwidth=2.0)
    o1, o2 = OK.KIFMM(one, 4), OK.KIFMM(two, 4)
    m2m, l2l, m2l, offs = ops.export(3), ops.export(4), ops.export(5), ops.export(6)
    for o in range(8):
        oc = ((o >> 2) & 1, (o >> 1) & 1, o & 1)
        np.testing.assert_allclose(m2m[o], o1.m2m(1, oc), rtol=1e-13)
        np.testing.assert_allclose(l2l[o], o2.l2l(1, oc), rtol=1e-13)
    assert len({tuple(v) for v in offs.astype(int)}) == 316
    for k in (0, 57, 315):
        np.testing.assert_allclose(m2l[k], o1.m2l(0, tuple(offs[k].astype(int))), rtol=1e-13)


def test_error_paths():
    x = np.random.default_rng(0).random((10, 3))
    with pytest.raises(K.KifmmError, match="EINVAL"):
        K.Operators(1)
    with pytest.raises(K.KifmmError, match="EINVAL"):
        K.Operators(17)
    with pytest.raises(K.KifmmError, match="EINVAL"):
        K.Operators(6, rcond=0.0)
    with pytest.raises(K.KifmmError, match="EINVAL"):
        K.Tree(np.zeros((0, 3)))
    bad = x.copy()
    bad[3, 1] = np.nan
    with pytest.raises(K.KifmmError, match="non-finite"):
        K.Tree(bad)
    bad[3, 1] = np.inf
    with pytest.raises(K.KifmmError, match="non-finite"):
        K.Tree(x, bad)
    with pytest.raises(K.KifmmError, match="ncrit"):
        K.Tree(x, ncrit=0)
    with pytest.raises(K.KifmmError, match="max_depth"):
        K.Tree(x, max_depth=21)
    with pytest.raises(K.KifmmError, match="uniform_depth"):
        K.Tree(x, uniform_depth=21)
    L = K.lib()
    import ctypes as C
    h = C.c_void_p()
    assert L.kifmm_build_tree(None, 10, None, 10, None, C.byref(h)) == 1
    t = K.Tree(x)
    ops = K.Operators(3)
    # evaluate argument errors are caught before any device work
    assert L.kifmm_evaluate(t.handle, ops.handle, None, 1, None, 1, 1, None) == 1
    assert b"null" in L.kifmm_last_error()
    assert L.kifmm_evaluate(t.handle, ops.handle, C.c_void_p(8), 0, C.c_void_p(8), 1, 1, None) == 1
    assert L.kifmm_evaluate(None, ops.handle, C.c_void_p(8), 1, C.c_void_p(8), 1, 1, None) == 1
    assert L.kifmm_evaluate(t.handle, ops.handle, C.c_void_p(8), 1, C.c_void_p(8), 1, 9, None) == 1
    assert L.kifmm_evaluate(t.handle, ops.handle, C.c_void_p(8), 65, C.c_void_p(8), 1, 1, None) == 4
    assert L.kifmm_tree_export_list(t.handle, 7, None, None) == 1


def test_tuning_keys_validated():
    """Every tuning key accepts its documented values and rejects others
    (host only: a value takes effect at the next evaluate)."""
    good = {"m2l_tile_cols": (64, 96, 128, 160, 192), "m2l_split": (0, 1), "m2l_pair_fill": (0, 40, 101),
            "near_fork": (0, 1, 2, 3, 4), "graph": (0, 1), "m2l_fp64_sum_min_p": (2, 10, 17),
            "m2l_check_min_p": (2, 10, 17), "far_fp64_min_p": (2, 10, 17), "m2l_wide": (0, 1),
            "m2l_rows": (0, 128, 160), "m2l_async": (0, 1)}
    bad = {"m2l_tile_cols": (0, 80, 256), "m2l_split": (2, -1), "m2l_pair_fill": (-1, 102),
           "near_fork": (-1, 5), "graph": (2,), "m2l_fp64_sum_min_p": (1, 18),
           "m2l_check_min_p": (1, 18), "far_fp64_min_p": (1, 18), "m2l_wide": (2, -1),
           "m2l_rows": (96, 1, -1), "m2l_async": (2, -1)}
    defaults = {"m2l_tile_cols": 64, "m2l_split": 1, "m2l_pair_fill": 40, "near_fork": 4, "graph": 1,
                "m2l_fp64_sum_min_p": 10, "m2l_check_min_p": 10, "far_fp64_min_p": 10, "m2l_wide": 0, "m2l_rows": 0,
                "m2l_async": 1}
    try:
        for k, vs in good.items():
            for v in vs:
                K.set_tuning(k, v)
        for k, vs in bad.items():
            for v in vs:
                with pytest.raises(K.KifmmError):
                    K.set_tuning(k, v)
        with pytest.raises(K.KifmmError, match="unknown"):
            K.set_tuning("no_such_key", 1)
    finally:
        for k, v in defaults.items():
            K.set_tuning(k, v)


def test_operator_cache_roundtrip_and_rejections(tmp_path):
    """kifmm_ops_save / kifmm_ops_load (host only): a saved cache loads back
    bitwise equal under its own key and is refused under another key, when
    damaged, truncated, foreign or missing."""
    ops = K.Operators(4)
    path = str(tmp_path / "ops4.bin")
    ops.save(path)
    back = K.Operators.load(path, 4)
    for which in range(7):
        np.testing.assert_array_equal(back.export(which), ops.export(which))
    with pytest.raises(K.KifmmError, match="another key"):
        K.Operators.load(path, 5)
    with pytest.raises(K.KifmmError, match="another key"):
        K.Operators.load(path, 4, rcond=1e-8)
    raw = bytearray(open(path, "rb").read())
    raw[len(raw) // 2] ^= 0x40
    bad = tmp_path / "damaged.bin"
    bad.write_bytes(bytes(raw))
    with pytest.raises(K.KifmmError, match="checksum"):
        K.Operators.load(str(bad), 4)
    short = tmp_path / "short.bin"
    short.write_bytes(open(path, "rb").read()[:1000])
    with pytest.raises(K.KifmmError, match="truncated"):
        K.Operators.load(str(short), 4)
    foreign = tmp_path / "foreign.bin"
    foreign.write_bytes(b"not an operator file at all")
    with pytest.raises(K.KifmmError, match="not an operator cache"):
        K.Operators.load(str(foreign), 4)
    with pytest.raises(K.KifmmError, match="cannot read"):
        K.Operators.load(str(tmp_path / "missing.bin"), 4)
    # the cache helper computes once, then loads
    a = K.Operators.cached(3, cache_dir=str(tmp_path))
    b = K.Operators.cached(3, cache_dir=str(tmp_path))
    np.testing.assert_array_equal(a.export(1), b.export(1))
    assert K.lib().kifmm_precompute_operators_ex(4, 1e-9, 2, None) == 1  # EINVAL


def test_screened_operators_and_update_arguments_on_host():
    """Host-side argument checks of the screened-kernel precompute and the
    point update (no device work is reached)."""
    import ctypes as C
    L = K.lib()
    h = C.c_void_p()
    assert L.kifmm_precompute_operators_screened(4, 1e-9, 0.0, 0.5, 4, 0, C.byref(h)) == 1   # kappa
    assert L.kifmm_precompute_operators_screened(4, 1e-9, 2.0, 0.0, 4, 0, C.byref(h)) == 1   # root
    assert L.kifmm_precompute_operators_screened(4, 1e-9, 2.0, 0.5, 1, 0, C.byref(h)) == 1   # max_level
    assert L.kifmm_precompute_operators_screened(4, 1e-9, 2.0, 0.5, 4, 8, C.byref(h)) == 1   # flag
    assert L.kifmm_precompute_operators_screened(4, 1e-9, 2.0, 0.5, 3, 0, C.byref(h)) == 0   # host SVD
    L.kifmm_ops_destroy(h)
    assert L.kifmm_tree_update_points(None, None, None, None) == 1
    x = np.random.default_rng(0).random((100, 3))
    t = K.Tree(x, uniform_depth=2, center=(0.5, 0.5, 0.5), halfwidth=0.5)
    assert L.kifmm_tree_update_points(t.handle, None, None, None) == 1


def test_screened_tables_match_oracle_per_level():
    """Screened-kernel tables (host precompute) against the oracle's operators,
    which it forms at each level from the actual box size: in the tables'
    units set l is r_l times the physical operator (the pseudo-inverses
    1 / r_l times), r_l = r0 / 2^l."""
    import ctypes as C
    p, kappa, r0, lmax = 4, 3.0, 1.0, 4
    h = C.c_void_p()
    K._check(K.lib().kifmm_precompute_operators_screened(p, 1e-9, kappa, r0, lmax, 0, C.byref(h)))
    ops = K.Operators(p, _handle=h)
    assert K.lib().kifmm_ops_levels(h) == lmax + 1
    uc2e, m2m, l2l, m2l, offs = ops.export(1), ops.export(3), ops.export(4), ops.export(5), ops.export(6)
    assert uc2e.shape == (lmax + 1, ops.n, ops.n) and np.all(uc2e[:2] == 0)
    tree = Octree(np.zeros((1, 3)), np.zeros((1, 3)), uniform_depth=0, center=(0, 0, 0), halfwidth=r0)
    o = OK.KIFMM(tree, p, kappa=kappa)
    for lev in (2, 4):
        r = r0 / 2 ** lev
        assert np.linalg.norm(uc2e[lev] - o.uc2e(lev) / r) / np.linalg.norm(o.uc2e(lev) / r) < 1e-9
        for k in (0, 123, 315):
            np.testing.assert_allclose(m2l[lev, k], r * o.m2l(lev, tuple(offs[k].astype(int))), rtol=1e-12)
        oc = (1, 0, 1)
        np.testing.assert_allclose(m2m[lev, 5], r * o.m2m(lev + 1, oc), rtol=1e-12)
        np.testing.assert_allclose(l2l[lev, 5], r * o.l2l(lev, oc), rtol=1e-12)


def test_injected_allocation_failures_on_the_host(tmp_path):
    """The allocation-failure hook (kifmm_debug_fail_allocations): a tree
    build, a precompute and a cache load fail with ENOMEM when their
    allocation point is hit, leave nothing behind, and work again once the
    hook has fired (it disarms itself)."""
    import ctypes as C
    L = K.lib()
    x, _ = I.uniform_cube(2000, seed=12)
    prm = K._params(2, 8, 4, True, (0.5, 0.5, 0.5), 0.5)
    h = C.c_void_p()
    K.fail_allocations_after(0)
    assert L.kifmm_build_tree(K._dptr(x), len(x), K._dptr(x), len(x), C.byref(prm), C.byref(h)) == 2
    assert b"injected" in L.kifmm_last_error() and not h.value
    t = K.Tree(x, uniform_depth=2, **CUBE)  # disarmed after firing
    assert t.info().n_src == 2000
    K.fail_allocations_after(0)
    with pytest.raises(K.KifmmError, match="ENOMEM"):
        K.Operators(3)
    ops = K.Operators(3)
    path = str(tmp_path / "ops.bin")
    ops.save(path)
    K.fail_allocations_after(0)
    with pytest.raises(K.KifmmError, match="ENOMEM"):
        K.Operators.load(path, 3)
    assert K.Operators.load(path, 3).n == ops.n
    K.fail_allocations_after(5)  # armed but not reached by the host build
    K.Tree(x, uniform_depth=2, **CUBE)
    K.fail_allocations_after(-1)
