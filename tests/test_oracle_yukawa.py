"""Pins for the oracle's screened (Yukawa) kernel exp(-kappa r) / (4 pi r),
the second kernel of the kernel-independent method (the paper's experiments
use the Laplace kernel only).

The direct sum is pinned by a closed form and by the PDE the kernel solves
away from its sources, Laplacian(phi) = kappa^2 phi (central differences);
the KIFMM with the screened kernel (operators formed per level from the
actual box sizes) by its convergence in p against the direct sum, for weak
and strong screening, on a uniform and an adaptive tree.
"""
import numpy as np

from oracle import direct, kifmm as OK
from oracle.octree import Octree
from paper_2303_08394_amd import inputs as I

CUBE = dict(center=(0.5, 0.5, 0.5), halfwidth=0.5)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_closed_form():
    # unit charge at the origin, target (1, 2, 2) at distance 3, kappa = 0.5:
    # exp(-1.5) / (4 pi 3) = exp(-1.5) / (12 pi)
    got = direct.direct(np.zeros((1, 3)), np.array([1.0]), np.array([[1.0, 2.0, 2.0]]), kappa=0.5)
    assert abs(got[0] - np.exp(-1.5) / (12.0 * np.pi)) < 1e-16
    assert direct.kernel_matrix(np.zeros((1, 3)), np.zeros((1, 3)), kappa=0.5)[0, 0] == 0.0


def test_screened_poisson_equation():
    rng = np.random.default_rng(8)
    src, q = rng.random((300, 3)), rng.uniform(-1, 1, 300)
    tgt = rng.random((40, 3)) + np.array([2.0, 0.0, 0.0])  # away from the sources
    kappa, h = 2.0, 1e-3
    phi = direct.direct(src, q, tgt, kappa=kappa)
    lap = -6.0 * phi
    for c in range(3):
        e = np.zeros(3)
        e[c] = h
        lap = lap + direct.direct(src, q, tgt + e, kappa=kappa) + direct.direct(src, q, tgt - e, kappa=kappa)
    lap /= h * h
    assert rel(lap, kappa ** 2 * phi) < 1e-5


def test_kifmm_converges_uniform():
    x, q = I.uniform_cube(3000, seed=1, charge_range=(-1, 1))
    tree = Octree(x, x, uniform_depth=3, **CUBE)
    for kappa in (1.0, 20.0):
        want = direct.direct(x, q[0], x, kappa=kappa)
        errs = [rel(OK.KIFMM(tree, p, kappa=kappa).evaluate(q[0]), want) for p in (4, 6)]
        # measured (kappa 1 / 20): 2.2e-4 / 2.4e-4 at p = 4, 2.4e-6 / 3.8e-6 at p = 6
        assert errs[0] < 5e-4 and errs[1] < 1e-5 and errs[1] < errs[0] / 30
    # the screened field differs from the Laplace one (the kernel is really applied)
    lap = OK.KIFMM(tree, 6).evaluate(q[0])
    assert rel(OK.KIFMM(tree, 6, kappa=1.0).evaluate(q[0]), lap) > 1e-2


def test_kifmm_adaptive():
    x, q = I.clustered(4000, seed=3)
    tree = Octree(x, x, ncrit=24, max_depth=10, **CUBE)
    got = OK.KIFMM(tree, 6, kappa=5.0).evaluate(q[0])
    assert rel(got, direct.direct(x, q[0], x, kappa=5.0)) < 5e-6  # measured 9.1e-7


def test_screened_gradient():
    """Gradient of the screened potential: central differences of the direct
    screened potential, and the KIFMM gradient against the direct one."""
    rng = np.random.default_rng(9)
    src, q = rng.random((300, 3)), rng.uniform(-1, 1, 300)
    tgt = rng.random((40, 3)) + np.array([2.0, 0.0, 0.0])
    kappa, h = 3.0, 1e-5
    g = direct.direct_gradient(src, q, tgt, kappa=kappa)
    for c in range(3):
        e = np.zeros(3)
        e[c] = h
        fd = (direct.direct(src, q, tgt + e, kappa=kappa) - direct.direct(src, q, tgt - e, kappa=kappa)) / (2 * h)
        assert rel(g[c], fd) < 1e-7
    x, qq = I.uniform_cube(3000, seed=1, charge_range=(-1, 1))
    tree = Octree(x, x, uniform_depth=3, **CUBE)
    pot, grad = OK.KIFMM(tree, 6, kappa=5.0).evaluate(qq[0], gradient=True)
    assert rel(grad, direct.direct_gradient(x, qq[0], x, kappa=5.0)) < 5e-5
