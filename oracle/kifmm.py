"""O2: the kernel-independent FMM evaluation in FP64, step by step.

Follows section "The Fast Multipole Method" (operators applied once per node
over a bottom-up then a top-down traversal), section "Computational structure
of FMM operators" (which operator reads which list; check potentials;
n_e = 6(p-1)^2 + 2) and section "Parallelization strategies for FMM
operators" (M2M/L2L translations scaled per level), with the KIFMM surfaces
of Ying et al. 2004 to which the paper defers.

Readings fixed here (the paper is silent on them):

* Check-to-equivalent solves use the pseudo-inverse truncated at a relative
  cutoff: singular values below rcond * sigma_max are dropped (default
  rcond = 1e-9).  UC2E = pinv(K(upward check, upward equivalent)),
  DC2E = pinv(K(downward check, downward equivalent)).
* Every operator matrix is formed for the level it is used at, from the
  actual box half-width r_l (no level-scaling shortcut): the scaling of the
  paper's M2M/L2L precomputation is checked against this in the tests.
* M2L runs on levels 2 .. depth (the V lists of levels 0 and 1 are empty);
  M2M is needed only up to level 2.
* Self-interaction (near field only): a source at distance zero from a target
  is skipped, as in Eq. (1).
* All arithmetic is FP64; summation order is free.

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import numpy as np

from .direct import gradient_matrices, kernel_matrix
from .octree import Octree
from .surface import RADIUS_INNER, RADIUS_OUTER, surface_grid


def pinv_truncated(a: np.ndarray, rcond: float) -> np.ndarray:
    """Pseudo-inverse from the SVD, dropping singular values < rcond * s_max."""
    u, s, vt = np.linalg.svd(a, full_matrices=False)
    keep = s >= rcond * s[0]
    return (vt[keep].T / s[keep]) @ u[:, keep].T


class KIFMM:
    """FP64 KIFMM on an oracle Octree at expansion order p."""

    def __init__(self, tree: Octree, p: int, rcond: float = 1e-9, kappa: float = 0.0):
        """kappa > 0: the screened (Yukawa) kernel exp(-kappa r) / (4 pi r)
        in every operator (the method is kernel independent; its operators
        are formed per level from the actual box sizes, which the screened
        kernel needs: it is not homogeneous)."""
        if p < 2:
            raise ValueError("p must be >= 2")
        self.tree = tree
        self.p = p
        self.rcond = rcond
        self.kappa = float(kappa)
        self.s = surface_grid(p)
        self.n = len(self.s)
        self._ops: dict = {}

    def _k(self, x, y):
        return kernel_matrix(x, y, self.kappa)

    # -- operators (one per level; translation-invariant ones keyed by offset)
    def _r(self, level):
        return self.tree.halfwidth(level)

    def uc2e(self, level):
        """Upward check potential -> upward equivalent density at `level`."""
        key = ("uc2e", level)
        if key not in self._ops:
            r = self._r(level)
            k = self._k(RADIUS_OUTER * r * self.s, RADIUS_INNER * r * self.s)
            self._ops[key] = pinv_truncated(k, self.rcond)
        return self._ops[key]

    def dc2e(self, level):
        """Downward check potential -> downward equivalent density at `level`."""
        key = ("dc2e", level)
        if key not in self._ops:
            r = self._r(level)
            k = self._k(RADIUS_INNER * r * self.s, RADIUS_OUTER * r * self.s)
            self._ops[key] = pinv_truncated(k, self.rcond)
        return self._ops[key]

    def _child_shift(self, child_level, octant):
        rc = self._r(child_level)
        return np.array([(2 * o - 1) * rc for o in octant], dtype=np.float64)

    def m2m(self, child_level, octant):
        """Child upward equivalent density -> parent upward check potential."""
        key = ("m2m", child_level, octant)
        if key not in self._ops:
            rp, rc = self._r(child_level - 1), self._r(child_level)
            x = RADIUS_OUTER * rp * self.s
            y = self._child_shift(child_level, octant) + RADIUS_INNER * rc * self.s
            self._ops[key] = self._k(x, y)
        return self._ops[key]

    def l2l(self, child_level, octant):
        """Parent downward equivalent density -> child downward check potential."""
        key = ("l2l", child_level, octant)
        if key not in self._ops:
            rp, rc = self._r(child_level - 1), self._r(child_level)
            x = self._child_shift(child_level, octant) + RADIUS_INNER * rc * self.s
            y = RADIUS_OUTER * rp * self.s
            self._ops[key] = self._k(x, y)
        return self._ops[key]

    def m2l(self, level, offset):
        """Source upward equivalent density -> target downward check potential,
        for a source box at (source - target) = offset boxes, same level."""
        key = ("m2l", level, offset)
        if key not in self._ops:
            r = self._r(level)
            x = RADIUS_INNER * r * self.s
            y = 2.0 * r * np.array(offset, dtype=np.float64) + RADIUS_INNER * r * self.s
            self._ops[key] = self._k(x, y)
        return self._ops[key]

    # -- surfaces of a box ---------------------------------------------------
    def _surf(self, b, radius):
        t = self.tree
        return t.center(b)[None, :] + (radius * self._r(t.level[b])) * self.s

    def _octant(self, b):
        t = self.tree
        pa = t.anchor[t.parent[b]]
        return tuple(t.anchor[b][d] - 2 * pa[d] for d in range(3))

    # -- evaluation ------------------------------------------------------------
    def evaluate(self, charges, sample=None, gradient=False):
        """Potentials at the tree's targets.

        charges: (n_src,) or (n_rhs, n_src) float64.
        sample: optional target indices; then only the leaves holding them
        (and their ancestors) run the downward pass, and only those targets
        are returned, in the order given.
        gradient: also return the gradient of the potential at the targets:
        the leaf stage (L2P, M2P, near field) applies the derivative of the
        kernel in the target position to the same densities and charges.
        Returns (n_tgt,) / (n_rhs, n_tgt), or (..., len(sample)); with
        gradient, the pair (potentials, gradients of shape (3, n_tgt) /
        (n_rhs, 3, n_tgt)).
        """
        t = self.tree
        q = np.asarray(charges, dtype=np.float64)
        one = q.ndim == 1
        qm = (q[None, :] if one else q).T          # (n_src, n_rhs)
        n_rhs = qm.shape[1]
        depth = t.depth
        nb = len(t.level)

        # Boxes whose downward pass is needed.
        if sample is None:
            tleaves = [b for b in t.leaves() if len(t.tgts[b])]
        else:
            sample = np.asarray(sample)
            want = set(sample.tolist())
            tleaves = [b for b in t.leaves() if any(int(i) in want for i in t.tgts[b])]
        need = set()
        for b in tleaves:
            a = b
            while a >= 0 and a not in need:
                need.add(a)
                a = t.parent[a]

        # Upward pass: P2M at leaves, M2M bottom-up (levels >= 2 only).
        up = {}
        for level in range(depth, 1, -1):
            for b in t.boxes_at(level):
                if t.is_leaf(b):
                    s_ids = t.srcs[b]
                    u = self._k(self._surf(b, RADIUS_OUTER), t.src[s_ids]) @ qm[s_ids]
                else:
                    u = np.zeros((self.n, n_rhs))
                    for c in t.children[b]:
                        u += self.m2m(level + 1, self._octant(c)) @ up[c]
                up[b] = self.uc2e(level) @ u

        # Downward pass: L2L, M2L (V), P2L (X), then DC2E, levels 2..depth.
        down = {}
        for level in range(2, depth + 1):
            for b in t.boxes_at(level):
                if b not in need:
                    continue
                d = np.zeros((self.n, n_rhs))
                par = t.parent[b]
                if par in down:
                    d += self.l2l(level, self._octant(b)) @ down[par]
                ab = t.anchor[b]
                for a in t.V(b):
                    off = tuple(t.anchor[a][k] - ab[k] for k in range(3))
                    d += self.m2l(level, off) @ up[a]
                x_dc = None
                for a in t.X(b):
                    if x_dc is None:
                        x_dc = self._surf(b, RADIUS_INNER)
                    s_ids = t.srcs[a]
                    d += self._k(x_dc, t.src[s_ids]) @ qm[s_ids]
                down[b] = self.dc2e(level) @ d

        # Leaves: L2P + M2P (W) + near field (U).
        pot = np.zeros((len(t.tgt), n_rhs))
        grad = np.zeros((3, len(t.tgt), n_rhs)) if gradient else None
        for b in tleaves:
            ids = t.tgts[b]
            x = t.tgt[ids]
            terms = []  # (sources, densities) seen by the leaf's targets
            if b in down:
                terms.append((self._surf(b, RADIUS_OUTER), down[b]))
            for a in t.W(b):
                terms.append((self._surf(a, RADIUS_INNER), up[a]))
            for a in t.U(b):
                s_ids = t.srcs[a]
                terms.append((t.src[s_ids], qm[s_ids]))
            acc = np.zeros((len(ids), n_rhs))
            for y, dens in terms:
                acc += self._k(x, y) @ dens
            pot[ids] = acc
            if gradient:
                for y, dens in terms:
                    g = gradient_matrices(x, y, self.kappa)
                    for c in range(3):
                        grad[c, ids] += g[c] @ dens
        out = pot.T
        if sample is not None:
            out = out[:, sample]
        if not gradient:
            return out[0] if one else out
        gout = grad.transpose(2, 0, 1)  # (n_rhs, 3, n_tgt)
        if sample is not None:
            gout = gout[:, :, sample]
        return (out[0], gout[0]) if one else (out, gout)


def kifmm(src, charges, tgt, p, *, uniform_depth=-1, ncrit=64, max_depth=12,
          balance=True, center=None, halfwidth=0.0, rcond=1e-9, sample=None, kappa=0.0):
    """Convenience wrapper: build the oracle tree, then evaluate (O2)."""
    tree = Octree(src, tgt, uniform_depth=uniform_depth, ncrit=ncrit,
                  max_depth=max_depth, balance=balance, center=center,
                  halfwidth=halfwidth)
    return KIFMM(tree, p, rcond, kappa).evaluate(charges, sample=sample)
