"""Pins for the oracle KIFMM (O2): operators against brute force, the
level scaling of the translation operators, error falling with p, invariances,
and planted mistakes that these pins must catch."""
import numpy as np
import pytest

from oracle import direct, kifmm
from oracle.direct import kernel_matrix
from oracle.octree import Octree
from oracle.surface import RADIUS_INNER, RADIUS_OUTER, surface_grid
from paper_2303_08394_amd import inputs as I

CUBE = dict(center=(0.5, 0.5, 0.5), halfwidth=0.5)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _box_ops(p, r=1.0):
    tree = Octree(np.zeros((1, 3)), np.zeros((1, 3)), uniform_depth=0,
                  center=(0, 0, 0), halfwidth=r)
    return kifmm.KIFMM(tree, p)


def test_pinv_matches_library():
    rng = np.random.default_rng(0)
    a = rng.normal(size=(40, 40)) @ np.diag(np.logspace(0, -14, 40)) @ rng.normal(size=(40, 40))
    np.testing.assert_allclose(kifmm.pinv_truncated(a, 1e-9),
                               np.linalg.pinv(a, rtol=1e-9), rtol=1e-6, atol=1e-6 * np.abs(np.linalg.pinv(a, rtol=1e-9)).max())


def _far_points(rng, n, rmin, rmax):
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    return d * rng.uniform(rmin, rmax, (n, 1))


def test_upward_equivalent_reproduces_check_and_far_field():
    rng = np.random.default_rng(1)
    y, q = rng.uniform(-1, 1, (300, 3)), rng.uniform(-1, 1, 300)
    far = _far_points(rng, 400, 3.0 * np.sqrt(3), 8.0)
    errs = []
    for p in (2, 4, 6, 8):
        ops = _box_ops(p)
        s = surface_grid(p)
        u = kernel_matrix(RADIUS_OUTER * s, y) @ q
        phi = ops.uc2e(0) @ u
        # the density reproduces the field on its check surface
        res = _rel(kernel_matrix(RADIUS_OUTER * s, RADIUS_INNER * s) @ phi, u)
        assert res < {2: 0.5, 4: 1e-3, 6: 1e-6, 8: 1e-8}[p]
        errs.append(_rel(kernel_matrix(far, RADIUS_INNER * s) @ phi, kernel_matrix(far, y) @ q))
    assert errs == sorted(errs, reverse=True) and errs[2] < 1e-5 and errs[3] < 1e-6


def test_downward_equivalent_reproduces_inner_field():
    rng = np.random.default_rng(2)
    # sources well outside the box (beyond 3 half-widths per axis)
    y = _far_points(rng, 300, 4.0 * np.sqrt(3), 9.0)
    q = rng.uniform(-1, 1, 300)
    x = rng.uniform(-1, 1, (400, 3))
    errs = []
    for p in (2, 4, 6, 8):
        ops = _box_ops(p)
        s = surface_grid(p)
        d = kernel_matrix(RADIUS_INNER * s, y) @ q
        phi = ops.dc2e(0) @ d
        errs.append(_rel(kernel_matrix(x, RADIUS_OUTER * s) @ phi, kernel_matrix(x, y) @ q))
    assert errs == sorted(errs, reverse=True) and errs[2] < 1e-5


def test_level_scaling_of_operators():
    """M2M/L2L/M2L and the check-to-equivalent solves scale with the level
    (the precompute-and-scale of section 'Parallelization strategies')."""
    ops = _box_ops(6, r=0.5)
    for l in (2, 3, 5):
        f = 2.0 ** l
        np.testing.assert_allclose(ops.uc2e(l) * f, ops.uc2e(0), rtol=0, atol=1e-6 * np.abs(ops.uc2e(0)).max())
        np.testing.assert_allclose(ops.m2l(l, (2, -3, 1)) / f, ops.m2l(0, (2, -3, 1)), rtol=1e-12)
        np.testing.assert_allclose(ops.m2m(l, (1, 0, 1)) / f, ops.m2m(1, (1, 0, 1)) / 2, rtol=1e-12)
        np.testing.assert_allclose(ops.l2l(l, (0, 1, 1)) / f, ops.l2l(1, (0, 1, 1)) / 2, rtol=1e-12)


def _uniform_case(n=4000, depth=3, seed=0, charge_range=(0.0, 1.0)):
    x, q = I.uniform_cube(n, seed=seed, charge_range=charge_range)
    return x, q[0], depth


def test_error_falls_with_p_uniform():
    x, q, depth = _uniform_case()
    ref = direct.direct(x, q, x)
    errs = [_rel(kifmm.kifmm(x, q, x, p, uniform_depth=depth, **CUBE), ref) for p in (2, 3, 4, 6, 8)]
    assert all(a > b for a, b in zip(errs, errs[1:])), errs
    assert errs[3] < 1e-5 and errs[4] < 1e-7


def test_error_adaptive_sphere_and_clusters():
    xs, qs = I.sphere_surface(5000, seed=0)
    ref = direct.direct(xs, qs[0], xs)
    t = Octree(xs, xs, ncrit=32, max_depth=8)
    e4 = _rel(kifmm.KIFMM(t, 4).evaluate(qs[0]), ref)
    e6 = _rel(kifmm.KIFMM(t, 6).evaluate(qs[0]), ref)
    assert e6 < e4 and e6 < 1e-5
    xc, qc = I.clustered(5000, seed=4, sigma=0.05)
    ref = direct.direct(xc, qc[0], xc)
    t = Octree(xc, xc, ncrit=24, max_depth=8, **CUBE)
    assert sum(len(t.W(b)) for b in t.leaves()) > 0
    assert _rel(kifmm.KIFMM(t, 6).evaluate(qc[0]), ref) < 1e-5


def test_invariances_and_multi_rhs():
    x, q, depth = _uniform_case(n=3000, charge_range=(-1.0, 1.0))
    base = kifmm.kifmm(x, q, x, 5, uniform_depth=depth, **CUBE)
    # homogeneity: x -> s x gives phi -> phi / s
    s = 3.0
    sc = kifmm.kifmm(s * x, q, s * x, 5, uniform_depth=depth, center=(1.5, 1.5, 1.5), halfwidth=1.5)
    assert _rel(sc, base / s) < 1e-8
    # translation invariance
    sh = kifmm.kifmm(x + 7.25, q, x + 7.25, 5, uniform_depth=depth, center=(7.75,) * 3, halfwidth=0.5)
    assert _rel(sh, base) < 1e-8
    # linearity and multiple right-hand sides in one call
    q2 = np.stack([q, np.ones_like(q), 2 * q - 1])
    m = kifmm.kifmm(x, q2, x, 5, uniform_depth=depth, **CUBE)
    # (the truncated pseudo-inverse amplifies rounding-order differences by
    # up to 1/rcond, so FP64 results agree to ~1e-9, not to machine epsilon)
    assert _rel(m[0], base) < 1e-8
    assert _rel(m[2], 2 * base - m[1]) < 1e-8
    # zero charges give zero potentials
    assert np.all(kifmm.kifmm(x, 0 * q, x, 3, uniform_depth=depth, **CUBE) == 0)


def test_single_charge_closed_form():
    rng = np.random.default_rng(4)
    src = np.array([[0.13, 0.71, 0.42]])
    tgt = rng.random((2000, 3))
    phi = kifmm.kifmm(src, np.array([1.0]), tgt, 6, uniform_depth=3, **CUBE)
    r = np.linalg.norm(tgt - src, axis=1)
    assert _rel(phi, 1 / (4 * np.pi * r)) < 1e-5


def test_sample_matches_full():
    x, q = I.clustered(3000, seed=11)
    t = Octree(x, x, ncrit=20, max_depth=8, **CUBE)
    fm = kifmm.KIFMM(t, 4)
    full = fm.evaluate(q[0])
    idx = I.sample_indices(3000, 50)
    np.testing.assert_allclose(fm.evaluate(q[0], sample=idx), full[idx], rtol=1e-13, atol=1e-13)


# --- planted mistakes: each must break at least one of the pins above -------

def _adaptive_err(monkeypatch=None):
    x, q = I.clustered(3000, seed=4, sigma=0.05)
    ref = direct.direct(x, q[0], x)
    t = Octree(x, x, ncrit=20, max_depth=8, **CUBE)
    return _rel(kifmm.KIFMM(t, 6).evaluate(q[0]), ref)


@pytest.mark.parametrize("mistake", ["drop_W", "drop_X", "drop_V", "transpose_m2l",
                                     "flip_m2l_offset", "uc2e_radius_mismatch", "drop_l2l",
                                     "m2m_wrong_octant"])
def test_planted_mistakes_are_caught(monkeypatch, mistake):
    assert _adaptive_err() < 1e-5
    if mistake == "drop_W":
        monkeypatch.setattr(Octree, "W", lambda self, b: [])
    elif mistake == "drop_X":
        monkeypatch.setattr(Octree, "X", lambda self, b: [])
    elif mistake == "drop_V":
        orig = Octree.V
        monkeypatch.setattr(Octree, "V", lambda self, b: orig(self, b)[1:])
    elif mistake == "transpose_m2l":
        orig = kifmm.KIFMM.m2l
        monkeypatch.setattr(kifmm.KIFMM, "m2l", lambda self, l, o: orig(self, l, o).T)
    elif mistake == "flip_m2l_offset":
        orig = kifmm.KIFMM.m2l
        monkeypatch.setattr(kifmm.KIFMM, "m2l", lambda self, l, o: orig(self, l, tuple(-v for v in o)))
    elif mistake == "uc2e_radius_mismatch":
        def bad(self, level):
            r = self._r(level)
            k = kernel_matrix(2.5 * r * self.s, RADIUS_INNER * r * self.s)
            return kifmm.pinv_truncated(k, self.rcond)
        monkeypatch.setattr(kifmm.KIFMM, "uc2e", bad)
    elif mistake == "drop_l2l":
        monkeypatch.setattr(kifmm.KIFMM, "l2l", lambda self, l, o: np.zeros((self.n, self.n)))
    elif mistake == "m2m_wrong_octant":
        orig = kifmm.KIFMM.m2m
        monkeypatch.setattr(kifmm.KIFMM, "m2m", lambda self, l, o: orig(self, l, tuple(1 - v for v in o)))
    assert _adaptive_err() > 1e-4
