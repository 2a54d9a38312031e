"""Check and equivalent surfaces (section "Computational structure of FMM
operators"; the KIFMM surfaces of Ying et al. 2004, sec. 3, to which the paper
defers).

The n_e = 6(p-1)^2 + 2 quadrature points of order p are the points of the
p x p x p lattice {-1 + 2i/(p-1)}^3 that lie on the boundary of the cube
[-1, 1]^3: p^3 - (p-2)^3 = 6(p-1)^2 + 2 of them.  The paper fixes the count;
the lattice-boundary reading is the one that reproduces it for every p.

For a box with centre c and half-width r the four surfaces are
    upward equivalent    c + RADIUS_INNER * r * s
    upward check         c + RADIUS_OUTER * r * s
    downward equivalent  c + RADIUS_OUTER * r * s
    downward check       c + RADIUS_INNER * r * s
The paper does not give the radii; 1.05 and 2.95 keep the inner surface
outside the box and the outer surface inside the region where a well
separated box (centre at distance >= 4r, nearest point at 3r) starts.

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import numpy as np

RADIUS_INNER = 1.05
RADIUS_OUTER = 2.95


def n_surface(p: int) -> int:
    """Number of surface points of order p: 6(p-1)^2 + 2."""
    return 6 * (p - 1) ** 2 + 2


def surface_grid(p: int) -> np.ndarray:
    """(n_surface(p), 3) points of the lattice boundary, lexicographic order."""
    if p < 2:
        raise ValueError("expansion order p must be >= 2")
    g = np.array([-1.0 + 2.0 * i / (p - 1) for i in range(p)])
    g[0], g[-1] = -1.0, 1.0
    pts = []
    for a in range(p):
        for b in range(p):
            for c in range(p):
                if a in (0, p - 1) or b in (0, p - 1) or c in (0, p - 1):
                    pts.append((g[a], g[b], g[c]))
    return np.array(pts, dtype=np.float64)
