"""The screened (Yukawa) kernel exp(-kappa r) / (4 pi r) through the whole
GPU path (operators per level, particle kernels with the exponential factor)
against the oracle's FP64 KIFMM with the same kernel.

Tolerances as for the Laplace kernel: FP64 1e-8, FP32 and split-precision M2L
1e-5 (relative L2 over all targets).
"""
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
TOL = {"fp64": 1e-8, "fp32": 1e-5, "bf16x3": 1e-5, "f16x3": 1e-5}
_want = {}

CASES = {
    "uniform8k_d3_p6_k5": lambda: (*I.uniform_cube(8000, seed=40, charge_range=(-1, 1)), 6, 5.0,
                                   dict(uniform_depth=3, **CUBE)),
    "clustered6k_nc24_p5_k2": lambda: (*I.clustered(6000, seed=41), 5, 2.0, dict(ncrit=24, max_depth=10, **CUBE)),
    "sphere8k_nc32_p5_k10": lambda: (*I.sphere_surface(8000, seed=42, jitter=0.0), 5, 10.0,
                                     dict(ncrit=32, max_depth=12)),
}


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu(tree, ops, q, precision):
    out = K.evaluate(tree, ops, torch.as_tensor(q, dtype=torch.float64, device=DEV), precision=precision)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3", "f16x3"])
def test_screened_vs_oracle(name, precision):
    x, q, p, kappa, kw = CASES[name]()
    tree = K.Tree(x, **kw)
    ops = K.Operators.screened(p, kappa, tree)
    got = gpu(tree, ops, q, precision)
    if name not in _want:
        _want[name] = OK.KIFMM(Octree(x, x, **kw), p, kappa=kappa).evaluate(q)
    e = rel(got, _want[name])
    print(f"{name} {precision}: {e:.2e}")
    assert e < TOL[precision]


def test_screened_batch_kernel_switch_and_errors(tmp_path):
    x1, q1 = I.uniform_cube(5000, seed=43)
    x2, q2 = I.clustered(4000, seed=44)
    t1 = K.Tree(x1, uniform_depth=3, **CUBE)
    t2 = K.Tree(x2, ncrit=32, max_depth=8, **CUBE)  # same root box
    ops = K.Operators.screened(5, 3.0, t2, max_level=8)
    qs = [torch.as_tensor(q[0], dtype=torch.float64, device=DEV) for q in (q1, q2)]
    outs = K.evaluate_batch([t1, t2], ops, qs, precision="fp32")
    torch.cuda.synchronize()
    for t, q, o in zip((t1, t2), (q1, q2), outs):
        np.testing.assert_array_equal(o.cpu().numpy(), gpu(t, ops, q, "fp32")[0])
    # the same tree with Laplace operators, before and after: plans rebuilt per kernel
    lap = K.Operators(5)
    a = gpu(t1, lap, q1, "fp32")
    s1 = gpu(t1, ops, q1, "fp32")
    np.testing.assert_array_equal(gpu(t1, lap, q1, "fp32"), a)
    assert rel(s1, a) > 1e-2
    # another root box, the cache: refused
    other = K.Tree(x1 * 0.5, uniform_depth=3, center=(0.25, 0.25, 0.25), halfwidth=0.25)
    with pytest.raises(K.KifmmError, match="root half-width"):
        gpu(other, ops, q1, "fp32")
    with pytest.raises(K.KifmmError, match="Laplace"):
        ops.save(str(tmp_path / "s.bin"))


@pytest.mark.parametrize("precision", ["fp64", "fp32", "f16x3"])
def test_screened_gradient_vs_oracle(precision):
    x, q, p, kappa, kw = CASES["sphere8k_nc32_p5_k10"]()
    tree = K.Tree(x, **kw)
    ops = K.Operators.screened(p, kappa, tree)
    got = K.evaluate_gradient(tree, ops, torch.as_tensor(q, dtype=torch.float64, device=DEV),
                              precision=precision)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    pot, grad = OK.KIFMM(Octree(x, x, **kw), p, kappa=kappa).evaluate(q, gradient=True)
    e = rel(got[:, 1:], grad)
    print(f"screened gradient {precision}: {e:.2e}")
    assert e < (1e-8 if precision == "fp64" else 2e-5)
    assert rel(got[:, 0], pot) < TOL[precision]
