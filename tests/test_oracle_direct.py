"""Pins for the oracle's direct sum O1 (Eq. 1) and its surfaces."""
import os

import numpy as np
import pytest
from scipy.spatial.distance import cdist

from oracle import direct, surface

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_three_charges_hand_worked():
    data = np.loadtxt(os.path.join(GOLDEN, "direct_three_charges.txt"))
    x, q, want = data[:, :3], data[:, 3], data[:, 4] / (4 * np.pi)
    got = direct.direct(x, q, x)
    np.testing.assert_allclose(got, want, rtol=1e-15)


def test_single_charge_closed_form():
    rng = np.random.default_rng(1)
    y = np.array([[0.3, -0.2, 0.7]])
    x = rng.normal(size=(50, 3))
    r = np.linalg.norm(x - y, axis=1)
    got = direct.direct(y, np.array([2.5]), x)
    np.testing.assert_allclose(got, 2.5 / (4 * np.pi * r), rtol=1e-14)


def test_two_charge_symmetry_and_self_exclusion():
    x = np.array([[0.1, 0.2, 0.3], [0.4, -0.5, 0.9]])
    phi = direct.direct(x, np.array([1.0, 1.0]), x)
    assert phi[0] == pytest.approx(phi[1], rel=1e-15)
    # the self term is excluded: each sees only the other charge
    r = np.linalg.norm(x[0] - x[1])
    assert phi[0] == pytest.approx(1 / (4 * np.pi * r), rel=1e-15)
    assert np.all(np.isfinite(direct.kernel_matrix(x, x)))
    assert direct.kernel_matrix(x, x)[0, 0] == 0.0


def test_against_cdist_and_linearity():
    rng = np.random.default_rng(2)
    src, tgt = rng.random((300, 3)), rng.random((200, 3))
    q = rng.uniform(-1, 1, (3, 300))
    got = direct.direct(src, q, tgt, chunk=37)
    want = (1 / (4 * np.pi * cdist(tgt, src))) @ q.T
    np.testing.assert_allclose(got, want.T, rtol=1e-12)
    # linearity in the charges
    np.testing.assert_allclose(direct.direct(src, 2 * q[0] - q[1], tgt),
                               2 * got[0] - got[1], rtol=1e-10, atol=1e-12)
    # homogeneity of degree -1
    np.testing.assert_allclose(direct.direct(3 * src, q[0], 3 * tgt), got[0] / 3, rtol=1e-12)


@pytest.mark.parametrize("p,n", [(2, 8), (3, 26), (4, 56), (6, 152), (8, 296), (10, 488), (12, 728)])
def test_surface_counts(p, n):
    s = surface.surface_grid(p)
    assert len(s) == n == surface.n_surface(p) == p ** 3 - (p - 2) ** 3
    assert np.all(np.max(np.abs(s), axis=1) == 1.0)
    assert len(np.unique(s, axis=0)) == n
    # every coordinate is a lattice value -1 + 2i/(p-1)
    lat = np.round((s + 1) * (p - 1) / 2)
    np.testing.assert_allclose(s, -1 + 2 * lat / (p - 1), atol=1e-15)


def test_surface_symmetry():
    s = surface.surface_grid(6)
    key = lambda a: set(map(tuple, np.round(a, 12)))
    base = key(s)
    assert key(-s) == base
    assert key(s[:, [1, 0, 2]]) == base
    assert key(s[:, [2, 1, 0]]) == base
    with pytest.raises(ValueError):
        surface.surface_grid(1)
