"""Octree and interaction lists for the oracle, written from their definitions.

Sections "The Fast Multipole Method" (root cube split recursively into 8),
"Computational structure of FMM operators" (n_crit leaf capacity, the U, V,
W, X lists, the 2:1 balance condition) and "Data-oriented design" (nodes
identified by a unique key; here a dict from (level, i, j, k) to a box id).

Readings fixed here (the paper is silent on them):

* Root.  Given (center, halfwidth) if halfwidth > 0, else the bounding cube of
  sources and targets: c0 = (min + max)/2 per axis, r0 = max extent / 2 times
  (1 + 2^-20); r0 = 0.5 if all points coincide.
* Partition.  Level l has boxes of half-width r0 / 2^l.  A point's level-l box
  index is clamp(floor(t * 2^l), 0, 2^l - 1) per axis with the FP64 fraction
  t = (x - (c0 - r0)) / (2 r0).  A point on an internal face goes to the upper box.
* Refinement.  Uniform tree: every non-empty box is split until level
  `uniform_depth`.  Adaptive tree: a box is split while it holds more than
  ncrit sources or more than ncrit targets and its level is below max_depth.
  Only non-empty children are created (a child is non-empty when it holds a
  source or a target).
* Balance (adaptive only, on by default).  Two leaves that touch (face, edge or
  corner) differ by at most one level: a leaf touching a leaf more than one
  level finer is split into its non-empty children, repeated until stable.
* Adjacency.  Two boxes are adjacent when their closed cubes intersect.
  Colleagues of B: the existing same-level boxes adjacent to B, B included.
* Lists (Ying et al. 2004, to which the paper defers):
    U(B), leaf B: every leaf adjacent to B, B included.
    V(B), level >= 2: children of the colleagues of B's parent not adjacent to B.
    W(B), leaf B: descendants A of B's colleagues with A not adjacent to B and
          A's parent adjacent to B.
    X(B): every leaf A with B in W(A).

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import numpy as np


class Octree:
    """A linear octree over sources and targets (float64 (n, 3) arrays)."""

    def __init__(self, src, tgt, *, uniform_depth: int = -1, ncrit: int = 64,
                 max_depth: int = 12, balance: bool = True, center=None,
                 halfwidth: float = 0.0):
        self.src = np.asarray(src, dtype=np.float64)
        self.tgt = np.asarray(tgt, dtype=np.float64)
        self.uniform_depth = uniform_depth
        self.ncrit = ncrit
        self.max_depth = max_depth if uniform_depth < 0 else uniform_depth
        if halfwidth and halfwidth > 0:
            self.c0 = np.asarray(center, dtype=np.float64).copy()
            self.r0 = float(halfwidth)
        else:
            allp = np.vstack([self.src, self.tgt])
            mn, mx = allp.min(axis=0), allp.max(axis=0)
            self.c0 = 0.5 * (mn + mx)
            r0 = 0.5 * float(np.max(mx - mn)) * (1.0 + 2.0 ** -20)
            self.r0 = r0 if r0 > 0 else 0.5
        self.lo = self.c0 - self.r0
        # FP64 fraction of the root cube per point and axis.
        self.ts = (self.src - self.lo) / (2.0 * self.r0)
        self.tt = (self.tgt - self.lo) / (2.0 * self.r0)

        self.level: list[int] = []
        self.anchor: list[tuple] = []
        self.parent: list[int] = []
        self.children: list[list[int]] = []
        self.srcs: list[np.ndarray] = []
        self.tgts: list[np.ndarray] = []
        self.key: dict[tuple, int] = {}

        root = self._add(0, (0, 0, 0), -1,
                         np.arange(len(self.src)), np.arange(len(self.tgt)))
        stack = [root]
        while stack:
            b = stack.pop()
            if self._wants_split(b):
                stack.extend(self._split(b))
        if uniform_depth < 0 and balance:
            self._balance()
        self._cache: dict = {}

    # -- construction ------------------------------------------------------
    def _add(self, level, anchor, parent, sids, tids):
        b = len(self.level)
        self.level.append(level)
        self.anchor.append(tuple(int(v) for v in anchor))
        self.parent.append(parent)
        self.children.append([])
        self.srcs.append(sids)
        self.tgts.append(tids)
        self.key[(level,) + self.anchor[b]] = b
        return b

    @staticmethod
    def point_index(t: np.ndarray, level: int) -> np.ndarray:
        """Level-`level` box index of points with root fractions t (clamped floor)."""
        n = 2 ** level
        return np.clip(np.floor(t * float(n)), 0, n - 1).astype(np.int64)

    def _wants_split(self, b) -> bool:
        if self.uniform_depth >= 0:
            return self.level[b] < self.uniform_depth
        return ((len(self.srcs[b]) > self.ncrit or len(self.tgts[b]) > self.ncrit)
                and self.level[b] < self.max_depth)

    def _split(self, b):
        l = self.level[b] + 1
        si = self.point_index(self.ts[self.srcs[b]], l)
        ti = self.point_index(self.tt[self.tgts[b]], l)
        new = []
        base = np.array(self.anchor[b]) * 2
        for ox in (0, 1):
            for oy in (0, 1):
                for oz in (0, 1):
                    a = base + np.array([ox, oy, oz])
                    sm = np.all(si == a, axis=1)
                    tm = np.all(ti == a, axis=1)
                    if sm.any() or tm.any():
                        c = self._add(l, a, b, self.srcs[b][sm], self.tgts[b][tm])
                        self.children[b].append(c)
                        new.append(c)
        return new

    def is_leaf(self, b) -> bool:
        return len(self.children[b]) == 0

    def _touching_keys(self, b, level):
        """Keys of the level-`level` cells (level <= level(b)) whose closed cube meets b's."""
        lb = self.level[b]
        s = 2 ** (lb - level)
        n = 2 ** level
        rng = []
        for d in range(3):
            i = self.anchor[b][d]
            lo = max(-(-i // s) - 1, 0)
            hi = min((i + 1) // s, n - 1)
            rng.append(range(lo, hi + 1))
        return [(level, x, y, z) for x in rng[0] for y in rng[1] for z in rng[2]]

    def _balance(self):
        changed = True
        while changed:
            changed = False
            leaves = [b for b in range(len(self.level)) if self.is_leaf(b)]
            for b in leaves:
                for l2 in range(self.level[b] - 2, -1, -1):
                    for k in self._touching_keys(b, l2):
                        a = self.key.get(k)
                        if a is not None and self.is_leaf(a):
                            self._split(a)
                            changed = True

    # -- geometry ----------------------------------------------------------
    def halfwidth(self, level) -> float:
        return self.r0 / 2.0 ** level

    def center(self, b) -> np.ndarray:
        r = self.halfwidth(self.level[b])
        return self.lo + (2.0 * np.array(self.anchor[b], dtype=np.float64) + 1.0) * r

    def adjacent(self, a, b) -> bool:
        """Closed cubes of boxes a and b intersect."""
        la, lb = self.level[a], self.level[b]
        L = max(la, lb)
        sa, sb = 2 ** (L - la), 2 ** (L - lb)
        for d in range(3):
            alo = self.anchor[a][d] * sa
            blo = self.anchor[b][d] * sb
            if max(alo, blo) > min(alo + sa, blo + sb):
                return False
        return True

    @property
    def depth(self) -> int:
        return max(self.level)

    def boxes_at(self, level):
        return [b for b in range(len(self.level)) if self.level[b] == level]

    def leaves(self):
        return [b for b in range(len(self.level)) if self.is_leaf(b)]

    # -- interaction lists -------------------------------------------------
    def colleagues(self, b):
        l = self.level[b]
        i, j, k = self.anchor[b]
        out = []
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    c = self.key.get((l, i + dx, j + dy, k + dz))
                    if c is not None:
                        out.append(c)
        return out

    def _uw(self, b):
        key = ("uw", b)
        if key in self._cache:
            return self._cache[key]
        u, w = [], []
        # Coarser or same-level leaves touching b (b itself included).
        for l2 in range(0, self.level[b] + 1):
            for k in self._touching_keys(b, l2):
                a = self.key.get(k)
                if a is not None and self.is_leaf(a):
                    u.append(a)
        # Finer boxes: descend the colleagues' subtrees.
        stack = [c for col in self.colleagues(b) if col != b for c in self.children[col]]
        while stack:
            a = stack.pop()
            if self.adjacent(a, b):
                if self.is_leaf(a):
                    u.append(a)
                else:
                    stack.extend(self.children[a])
            else:
                w.append(a)
        self._cache[key] = (sorted(u), sorted(w))
        return self._cache[key]

    def U(self, b):
        """Near-field list of leaf b."""
        return self._uw(b)[0] if self.is_leaf(b) else []

    def W(self, b):
        """M2P list of leaf b."""
        return self._uw(b)[1] if self.is_leaf(b) else []

    def V(self, b):
        """M2L list of box b (empty above level 2)."""
        if self.level[b] < 2:
            return []
        key = ("v", b)
        if key not in self._cache:
            out = []
            for pc in self.colleagues(self.parent[b]):
                for a in self.children[pc]:
                    if not self.adjacent(a, b):
                        out.append(a)
            self._cache[key] = sorted(out)
        return self._cache[key]

    def X(self, b):
        """P2L list of box b: leaves a with b in W(a).

        b is in W(a) exactly when a is a leaf coarser than b that touches
        b's parent but not b (then every ancestor of b below a's level
        touches a and is split, so the W descent of a reaches b).
        """
        if self.level[b] < 1:
            return []
        key = ("x", b)
        if key not in self._cache:
            p = self.parent[b]
            out = []
            for l2 in range(0, self.level[b]):
                for k in self._touching_keys(p, l2):
                    a = self.key.get(k)
                    if a is not None and self.is_leaf(a) and not self.adjacent(a, b):
                        out.append(a)
            self._cache[key] = sorted(out)
        return self._cache[key]
