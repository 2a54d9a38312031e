"""Pins for the oracle's gradient of the potential (the derivative of Eq. (1)
in the target position; the paper evaluates potentials only).

The direct gradient is pinned by a closed form, by central differences of
the direct potential (O(h^2) accurate), by the pairwise antisymmetry of the
forces (sum_i q_i grad phi(x_i) = 0 for targets = sources) and by the
exclusion of coincident pairs.  The KIFMM gradient is pinned against the
direct gradient: its error falls with p like the potential's, on a uniform
tree and on an adaptive one with W and X lists (M2P and P2L terms).
"""
import numpy as np
import pytest

from oracle import direct, kifmm as OK
from oracle.octree import Octree
from paper_2303_08394_amd import inputs as I

CUBE = dict(center=(0.5, 0.5, 0.5), halfwidth=0.5)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_single_source_closed_form():
    # unit charge at the origin, target (1, 2, 2) at distance 3:
    # grad phi = -(1, 2, 2) / (4 pi 27) = -(1, 2, 2) / (108 pi)
    g = direct.direct_gradient(np.zeros((1, 3)), np.array([1.0]), np.array([[1.0, 2.0, 2.0]]))
    np.testing.assert_allclose(g[:, 0], -np.array([1.0, 2.0, 2.0]) / (108.0 * np.pi), rtol=1e-15)


def test_central_differences_of_the_potential():
    rng = np.random.default_rng(3)
    # targets apart from the sources (a unit cube away), where the potential is smooth
    src, tgt = rng.random((400, 3)), rng.random((60, 3)) + np.array([2.0, 0.0, 0.0])
    q = rng.uniform(-1, 1, (2, 400))
    g = direct.direct_gradient(src, q, tgt, chunk=17)
    h = 1e-5
    for c in range(3):
        e = np.zeros(3)
        e[c] = h
        fd = (direct.direct(src, q, tgt + e) - direct.direct(src, q, tgt - e)) / (2 * h)
        assert rel(g[:, c], fd) < 1e-7


def test_forces_cancel_and_self_pairs_excluded():
    rng = np.random.default_rng(4)
    x = rng.random((500, 3))
    q = rng.uniform(-1, 1, 500)
    g = direct.direct_gradient(x, q, x)
    net = (q[None, :] * g).sum(axis=1)          # sum_i q_i grad phi(x_i)
    scale = (np.abs(q)[None, :] * np.abs(g)).sum(axis=1)
    assert np.all(np.abs(net) < 1e-12 * scale)
    gm = direct.gradient_matrices(x[:5], x[:5])
    assert np.all(np.isfinite(gm)) and np.all(gm[:, range(5), range(5)] == 0.0)


def test_kifmm_gradient_converges_uniform():
    x, q = I.uniform_cube(3000, seed=1, charge_range=(-1, 1))
    want = direct.direct_gradient(x, q[0], x)
    tree = Octree(x, x, uniform_depth=3, **CUBE)
    errs = []
    for p in (4, 6, 8):
        pot, g = OK.KIFMM(tree, p).evaluate(q[0], gradient=True)
        errs.append(rel(g, want))
        if p == 6:  # the potential is the plain evaluation's
            np.testing.assert_array_equal(pot, OK.KIFMM(tree, p).evaluate(q[0]))
    # measured 4.4e-4, 9.1e-6, 2.8e-7
    assert errs[0] < 1e-3 and errs[1] < 3e-5 and errs[2] < 1e-6
    assert errs[1] < errs[0] / 10 and errs[2] < errs[1] / 10


def test_kifmm_gradient_adaptive_with_w_and_x_lists():
    x, q = I.clustered(4000, seed=3)
    tree = Octree(x, x, ncrit=24, max_depth=10, **CUBE)
    assert sum(len(tree.W(b)) for b in range(len(tree.level))) > 0
    assert sum(len(tree.X(b)) for b in range(len(tree.level))) > 0
    qm = np.vstack([q[0], np.random.default_rng(5).uniform(-1, 1, 4000)])
    pot, g = OK.KIFMM(tree, 6).evaluate(qm, gradient=True)
    assert g.shape == (2, 3, 4000)
    assert rel(g, direct.direct_gradient(x, qm, x)) < 5e-5  # measured 1.3e-5 (first column)
    # a sample returns the same targets' values
    idx = np.array([7, 3000, 11])
    ps, gs = OK.KIFMM(tree, 6).evaluate(qm, sample=idx, gradient=True)
    np.testing.assert_allclose(gs, g[:, :, idx], rtol=1e-12, atol=0)
