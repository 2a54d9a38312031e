"""FP64 CPU oracle for the 3D Laplace kernel-independent FMM evaluation.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import or call anything here.
The product path (the HIP library and its Python binding) never does, and
the oracle never imports the product package: the two share no code.

Contents
--------
direct   O1: the Laplace potential of Eq. (1) summed directly (definition), and
         its gradient in the target position (derivative of the same sum).
surface  the check / equivalent surface quadrature points (section "Computational
         structure of FMM operators": n_e = 6(p-1)^2 + 2).
octree   the octree (uniform, adaptive, 2:1 balanced) and the U, V, W, X
         interaction lists (same section), written from their definitions.
kifmm    O2: the KIFMM evaluation in FP64, step by step: P2M, M2M, M2L, P2L,
         L2L, L2P, M2P and the near field (section "The Fast Multipole Method");
         optionally the gradient, from the kernel's derivative in the leaf stage;
         optionally the screened (Yukawa) kernel exp(-kappa r) / (4 pi r).

Parity status: every function is pinned by the CPU tests in
``tests/test_oracle_*.py`` (closed forms, brute force, invariants, exact
integer counts).  No function is "parity unpinned".
"""
from . import direct, surface, octree, kifmm  # noqa: F401
