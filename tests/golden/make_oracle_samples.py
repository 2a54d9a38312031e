"""Writes the FP64 oracle's values on seeded target samples of the larger
parity workloads (tests/golden/oracle_<case>.npz).

The oracle (O2, the plain FP64 KIFMM of oracle/kifmm.py) is exact only to its
own arithmetic, and at these sizes it takes from seconds to minutes; the GPU
tests compare the HIP path with these stored values instead of re-running it.
Every value here comes from oracle/ alone, on inputs drawn by the seeded
recipes of paper_2303_08394_amd/inputs.py (random draws only, none of the
method's arithmetic).  Each file records

  idx          the sampled target indices (inputs.sample_indices),
  pot          the oracle potentials at them, [n_rhs][len(idx)],
  grad         (gradient cases) the oracle gradients, [n_rhs][3][len(idx)],
  inputs_sha   SHA-256 of the points and charges the recipe drew,
  oracle_sha   SHA-256 of the oracle's source files when the values were made,

and tests/test_oracle_samples.py checks on the CPU that both hashes still
match (a changed recipe or oracle makes the stored values stale: rerun this
script).  Usage: python tests/golden/make_oracle_samples.py [case ...]
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import kifmm as OK  # noqa: E402
from oracle.octree import Octree  # noqa: E402
from paper_2303_08394_amd import inputs as I  # noqa: E402

CUBE = dict(center=I.UNIT_CUBE_CENTER, halfwidth=I.UNIT_CUBE_HALFWIDTH)


def _uniform1m():
    prob = I.uniform_1m()
    return prob.points, prob.charges


# name: (inputs, order p, oracle tree arguments, sample size, with gradient)
CASES = {
    # twin of the multi-RHS workload at p = 10: 4,681 boxes x 4 right-hand
    # sides, >= 128 GEMM tiles per plan, so the FP64-sum M2L, the FP64
    # surface terms and the check-form M2L all run at their defaults
    "uniform100k_d4_p10_rhs4": (lambda: I.uniform_cube(100_000, seed=50, charge_range=(-1.0, 1.0), n_rhs=4),
                                10, dict(uniform_depth=4, **CUBE), 400, False),
    # twin of the 4M jittered sphere at p = 8 (adaptive, n_crit 64): its M2L
    # runs pair by pair; also the gradient on a jittered surface
    "sphere300k_nc64_p8": (lambda: I.sphere_surface(300_000, seed=40), 8, dict(ncrit=64, max_depth=12), 400, True),
    # the headline workload itself: 1M uniform-cube points, p = 6, depth 5
    "uniform1m_d5_p6": (_uniform1m, 6, dict(uniform_depth=5, **CUBE), 2000, False),
}


def inputs_sha(x: np.ndarray, q: np.ndarray) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(x, dtype=np.float64).tobytes())
    h.update(np.ascontiguousarray(q, dtype=np.float64).tobytes())
    return h.hexdigest()


def oracle_sha() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "oracle")
    for f in sorted(os.listdir(d)):
        if f.endswith(".py"):
            h.update(f.encode())
            with open(os.path.join(d, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def path(name: str) -> str:
    return os.path.join(HERE, f"oracle_{name}.npz")


def make(name: str) -> None:
    make_inputs, p, kw, k, grad = CASES[name]
    x, q = make_inputs()
    q = np.atleast_2d(q)
    t0 = time.time()
    tree = Octree(x, x, **kw)
    idx = I.sample_indices(len(x), k)
    res = OK.KIFMM(tree, p).evaluate(q, sample=idx, gradient=grad)
    out = dict(idx=idx, inputs_sha=inputs_sha(x, q), oracle_sha=oracle_sha(), p=p)
    if grad:
        out["pot"], out["grad"] = res
    else:
        out["pot"] = res
    np.savez(path(name), **out)
    print(f"{name}: {len(idx)} targets, {q.shape[0]} rhs, {time.time() - t0:.1f} s")


if __name__ == "__main__":
    for n in (sys.argv[1:] or list(CASES)):
        make(n)
