"""Operator precomputation with the pseudo-inverses on the GPU
(kifmm_precompute_operators_ex with KIFMM_PRECOMPUTE_DEVICE_SVD) against the
host's one-sided Jacobi path and the oracle.

The two SVD algorithms differ, so the pseudo-inverses agree only to the
conditioning of the kept singular values (cond up to 1/rcond = 1e9): the
tables are compared loosely, and the evaluation they feed at the FP64 floor
of section-4 parity (1e-8 relative L2), against the oracle and against the
host-precomputed operators.
"""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import kifmm as OK  # noqa: E402
from oracle.octree import Octree  # noqa: E402
from paper_2303_08394_amd import inputs as I  # noqa: E402
from paper_2303_08394_amd import kifmm as K  # noqa: E402

DEV = "cuda:0"
CUBE = dict(center=(0.5, 0.5, 0.5), halfwidth=0.5)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("p", [4, 6, 8])
def test_device_svd_operators(p):
    host = K.Operators(p)
    dev = K.Operators(p, device_svd=True)
    for which in (0, 3, 4, 5, 6):  # tables without a pseudo-inverse: identical
        np.testing.assert_array_equal(dev.export(which), host.export(which))
    for which in (1, 2):  # UC2E, DC2E
        e = rel(dev.export(which), host.export(which))
        print(f"p={p} table {which}: rel diff {e:.2e}")
        assert e < 1e-5
    x, q = I.uniform_cube(8000, seed=5, charge_range=(-1, 1))
    tree = K.Tree(x, uniform_depth=3, **CUBE)
    qd = torch.as_tensor(q, dtype=torch.float64, device=DEV)
    a = K.evaluate(tree, dev, qd, precision="fp64").cpu().numpy()
    b = K.evaluate(tree, host, qd, precision="fp64").cpu().numpy()
    want = OK.KIFMM(Octree(x, x, uniform_depth=3, **CUBE), p).evaluate(q)
    print(f"p={p}: device-SVD vs host-SVD {rel(a, b):.2e}, vs oracle {rel(a, want):.2e}")
    assert rel(a, b) < 1e-8
    assert rel(a, want) < 1e-8


def test_device_svd_time_and_cache_p10(tmp_path):
    t0 = time.perf_counter()
    dev = K.Operators(10, device_svd=True)
    t1 = time.perf_counter()
    path = str(tmp_path / "p10.bin")
    dev.save(path)
    t2 = time.perf_counter()
    back = K.Operators.load(path, 10)
    t3 = time.perf_counter()
    print(f"p=10: precompute with GPU SVD {t1 - t0:.2f} s, save {t2 - t1:.2f} s, load {t3 - t2:.2f} s")
    np.testing.assert_array_equal(back.export(1), dev.export(1))
