"""The stored oracle samples (tests/golden/oracle_*.npz, written by
tests/golden/make_oracle_samples.py from oracle/ alone) are current and are
what they claim to be:

* the seeded recipes still draw the inputs the values were computed for, and
  the oracle's source is unchanged since (else the values are stale);
* the stored potentials are a KIFMM of those inputs: against the direct sum
  of Eq. (1) (O1, the definition) on the sampled targets they differ by the
  truncation error of their order p, and no more (measured on these inputs:
  2.4e-6 at p = 6, 3.7e-9 at p = 8, 4.5-6.4e-9 at p = 10; a dropped or
  mis-indexed term of any list moves them by orders of magnitude);
* the stored gradients agree with the direct gradient likewise (4.6e-7 at
  p = 8).
"""
import os
import sys

import numpy as np
import pytest

from oracle import direct

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
import make_oracle_samples as M  # noqa: E402

# direct-sum bound on the stored FMM values, by order p
BOUND = {6: 1e-5, 8: 5e-8, 10: 5e-8}
GRAD_BOUND = {8: 2e-6}


def load(name):
    return dict(np.load(M.path(name)))


@pytest.mark.parametrize("name", list(M.CASES))
def test_sample_is_current_and_pinned(name):
    d = load(name)
    make_inputs, p, kw, k, grad = M.CASES[name]
    x, q = make_inputs()
    q = np.atleast_2d(q)
    assert str(d["inputs_sha"]) == M.inputs_sha(x, q), "recipe changed: rerun make_oracle_samples.py"
    assert str(d["oracle_sha"]) == M.oracle_sha(), "oracle changed: rerun make_oracle_samples.py"
    idx = d["idx"]
    assert len(idx) == k and int(d["p"]) == p
    assert d["pot"].shape == (q.shape[0], k)
    # the first targets of the sample against the definition
    sub = idx[:60]
    for r in range(q.shape[0]):
        want = direct.direct(x, q[r], x[sub], chunk=8)
        e = np.linalg.norm(d["pot"][r, :60] - want) / np.linalg.norm(want)
        assert e < BOUND[p], (r, e)
    if grad:
        want = direct.direct_gradient(x, q[0], x[sub], chunk=8)
        e = np.linalg.norm(d["grad"][0, :, :60] - want) / np.linalg.norm(want)
        assert e < GRAD_BOUND[p], e
