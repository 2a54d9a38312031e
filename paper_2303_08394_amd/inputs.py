"""Seeded synthetic workloads for the Laplace KIFMM evaluation.

This module only draws random numbers: it holds none of the method's
arithmetic and is shared by the tests, the oracle checks and the benchmark.

The paper measures on random point clouds only (uniform particles on a sphere
surface, section "Parallelization strategies for FMM operators"); the recipes
below add the uniform-cube, clustered, batched and multi-right-hand-side
shapes of the evaluation workloads.  Every recipe uses
``numpy.random.default_rng(seed)`` and draws its variables in the order they
are listed: positions first, then charges.
"""
from __future__ import annotations

import dataclasses

import numpy as np

UNIT_CUBE_CENTER = (0.5, 0.5, 0.5)
UNIT_CUBE_HALFWIDTH = 0.5


@dataclasses.dataclass
class Problem:
    """One evaluation problem: sources = targets, charges [n_rhs][n]."""

    points: np.ndarray          # (n, 3) float64, sources and targets
    charges: np.ndarray         # (n_rhs, n) float64
    p: int                      # expansion order
    uniform_depth: int          # >= 0: uniform tree; -1: adaptive
    ncrit: int                  # adaptive leaf capacity (ignored if uniform)
    max_depth: int              # adaptive depth cap
    center: tuple | None        # root centre, None = derived from the points
    halfwidth: float            # root half-width, 0 = derived
    name: str = ""

    @property
    def n(self) -> int:
        return self.points.shape[0]


def _rng(seed_or_rng):
    if isinstance(seed_or_rng, np.random.Generator):
        return seed_or_rng
    return np.random.default_rng(seed_or_rng)


def uniform_cube(n: int, seed=0, charge_range=(0.0, 1.0), n_rhs: int = 1):
    """Points i.i.d. uniform in [0,1)^3, then charges uniform in charge_range."""
    rng = _rng(seed)
    x = rng.random((n, 3))
    lo, hi = charge_range
    if n_rhs == 1:
        q = rng.uniform(lo, hi, n)[None, :] if (lo, hi) != (0.0, 1.0) else rng.random(n)[None, :]
    else:
        q = rng.uniform(lo, hi, (n_rhs, n))
    return x, q


def sphere_surface(n: int, seed=0, jitter: float = 1e-3):
    """Unit-sphere points: Gaussian directions normalised, radius 1 + N(0, jitter)."""
    rng = _rng(seed)
    g = rng.standard_normal((n, 3))
    u = g / np.linalg.norm(g, axis=1)[:, None]
    x = u * (1.0 + rng.normal(0.0, jitter, n))[:, None]
    q = rng.random(n)[None, :]
    return x, q


def clustered(n: int, seed=0, n_clusters: int = 8, sigma: float = 0.05):
    """Points around n_clusters Gaussian centres in [0.2,0.8)^3, kept inside [0,1)^3."""
    rng = _rng(seed)
    centers = rng.uniform(0.2, 0.8, (n_clusters, 3))
    out = np.empty((n, 3))
    filled = 0
    while filled < n:
        m = n - filled
        lab = rng.integers(n_clusters, size=m)
        pts = centers[lab] + rng.normal(0.0, sigma, (m, 3))
        ok = np.all((pts >= 0.0) & (pts < 1.0), axis=1)
        pts = pts[ok]
        out[filled:filled + len(pts)] = pts
        filled += len(pts)
    q = rng.random(n)[None, :]
    return out, q


# ---------------------------------------------------------------------------
# The five evaluation workloads (full size) and their small parity-test twins.
# ---------------------------------------------------------------------------

def plain_fp64_20k(n: int = 20_000) -> Problem:
    """N=20k uniform cube, charges [0,1), p=6, uniform depth 3, seed 0."""
    x, q = uniform_cube(n, seed=0)
    return Problem(x, q, p=6, uniform_depth=3, ncrit=0, max_depth=0,
                   center=UNIT_CUBE_CENTER, halfwidth=UNIT_CUBE_HALFWIDTH,
                   name=f"uniform_cube_n{n}_p6_depth3")


def uniform_1m(n: int = 1_000_000, depth: int = 5) -> Problem:
    """N=1M uniform cube, charges [-1,1), p=6, uniform depth 5, seed 0."""
    x, q = uniform_cube(n, seed=0, charge_range=(-1.0, 1.0))
    return Problem(x, q, p=6, uniform_depth=depth, ncrit=0, max_depth=0,
                   center=UNIT_CUBE_CENTER, halfwidth=UNIT_CUBE_HALFWIDTH,
                   name=f"uniform_cube_n{n}_p6_depth{depth}")


def sphere_4m(n: int = 4_000_000, ncrit: int = 64, max_depth: int = 12) -> Problem:
    """N=4M sphere surface, charges [0,1), p=8, adaptive ncrit=64, root from data."""
    x, q = sphere_surface(n, seed=0)
    return Problem(x, q, p=8, uniform_depth=-1, ncrit=ncrit, max_depth=max_depth,
                   center=None, halfwidth=0.0, name=f"sphere_n{n}_p8_ncrit{ncrit}")


def batch_problem(k: int, scale: float = 1.0) -> Problem:
    """Problem k of the 64-problem batch: N log-uniform in [1e4, 5e5] (times scale);
    k < 32 uniform cube, k >= 32 eight Gaussian clusters; p=6, ncrit=64."""
    rng = np.random.default_rng(k)
    n = int(round(np.exp(rng.uniform(np.log(1e4), np.log(5e5))) * scale))
    n = max(n, 16)
    if k < 32:
        x, q = uniform_cube(n, seed=rng)
    else:
        x, q = clustered(n, seed=rng)
    return Problem(x, q, p=6, uniform_depth=-1, ncrit=64, max_depth=12,
                   center=UNIT_CUBE_CENTER, halfwidth=UNIT_CUBE_HALFWIDTH,
                   name=f"batch{k}_n{n}")


def multi_rhs_1m(n: int = 1_000_000, n_rhs: int = 32, depth: int = 5, p: int = 10) -> Problem:
    """N=1M uniform cube with n_rhs charge vectors in [-1,1); p=10, depth 5."""
    x, q = uniform_cube(n, seed=0, charge_range=(-1.0, 1.0), n_rhs=n_rhs)
    return Problem(x, q, p=p, uniform_depth=depth, ncrit=0, max_depth=0,
                   center=UNIT_CUBE_CENTER, halfwidth=UNIT_CUBE_HALFWIDTH,
                   name=f"uniform_cube_n{n}_rhs{n_rhs}_p{p}_depth{depth}")


def paper_sphere_1m(n: int = 1_000_000, ncrit: int = 150, p: int = 6) -> Problem:
    """The paper's experiment shape: N=1M points on the unit sphere surface
    (no radial jitter), charges [0,1), p=6, adaptive ncrit=150, root from data."""
    x, q = sphere_surface(n, seed=0, jitter=0.0)
    return Problem(x, q, p=p, uniform_depth=-1, ncrit=ncrit, max_depth=16,
                   center=None, halfwidth=0.0, name=f"sphere_surface_n{n}_p{p}_ncrit{ncrit}")


def sample_indices(n: int, k: int, seed: int = 12345) -> np.ndarray:
    """A sorted seeded subsample of k distinct indices out of n."""
    rng = np.random.default_rng(seed)
    k = min(k, n)
    return np.sort(rng.choice(n, size=k, replace=False))
