"""GPU parity with the FP64 oracle on the code paths the measured workloads
run, through the C ABI (element by element on seeded target samples of the
oracle; the values come from tests/golden/make_oracle_samples.py, which
calls oracle/ alone; tests/test_oracle_samples.py pins them).

* p = 10 twin of the multi-RHS workload (100k uniform points, depth 4, four
  right-hand sides): >= 128 GEMM tiles per plan, so the M2L with FP64 step
  sums, the FP64 equivalent-surface terms and the check-form M2L run at their
  default orders.  Gates: FP64 1e-8; FP16x3 and the FP64-bulk mixed modes
  1e-6 (the multi-RHS accuracy target, which these modes serve); FP32, BF16x3
  and BF16x5 1e-5 (their BF16 operator parts keep 16 significant bits:
  BF16x5 measured 2.0e-6 here, BF16x3 ~7e-6 at this order).
* p = 8 twin of the 4M jittered sphere (300k points, adaptive, n_crit 64):
  M2L pair by pair (the default for such trees) and with 128-column tiles
  forced as in the autotuned 4M run.  Gates: FP64 1e-8, mixed 1e-5.
* the headline workload itself (1M points, p = 6, depth 5) on 2,000 sampled
  targets, every mode.  Gates: FP64 1e-8, mixed 1e-5.
The FP64 gate is set by the two sides' different SVD drivers (the truncated
pseudo-inverses agree to ~1e-8 relative at rcond = 1e-9; measured FP64
parity 1e-12 .. 2e-9 on the small cases).
"""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2303_08394_amd import inputs as I  # noqa: E402
from paper_2303_08394_amd import kifmm as K  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
import make_oracle_samples as M  # noqa: E402

DEV = "cuda:0"
MODES = ["fp64", "fp32", "bf16x3", "bf16x5", "f16x3", "fp64+m2l_fp32", "fp64+m2l_f16x3"]
_cache = {}


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def case(name):
    """(tree, ops, device charges, stored oracle sample) of a stored case."""
    if name not in _cache:
        make_inputs, p, kw, k, grad = M.CASES[name]
        x, q = make_inputs()
        q = np.atleast_2d(q)
        d = dict(np.load(M.path(name)))
        assert str(d["inputs_sha"]) == M.inputs_sha(x, q)
        tree = K.Tree(x, uniform_depth=kw.get("uniform_depth", -1), ncrit=kw.get("ncrit", 64),
                      max_depth=kw.get("max_depth", 12), center=kw.get("center"),
                      halfwidth=kw.get("halfwidth", 0.0))
        ops = K.Operators(p, device_svd=p >= 10)
        qd = torch.as_tensor(q, dtype=torch.float64, device=DEV)
        _cache[name] = (tree, ops, qd, d)
    return _cache[name]


def eval_side_stream(tree, ops, qd, precision):
    """Evaluation as bench.py times it: captured on a side stream, replayed;
    the replay must equal the capture bitwise."""
    out = torch.empty(qd.shape, dtype=torch.float64, device=DEV)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        K.evaluate(tree, ops, qd, precision=precision, out=out)
        torch.cuda.synchronize()
        first = out.cpu().numpy().copy()
        K.evaluate(tree, ops, qd, precision=precision, out=out)
        torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), first)
    return first


def check(name, precision, tol):
    tree, ops, qd, d = case(name)
    got = eval_side_stream(tree, ops, qd, precision)[:, d["idx"]]
    e = rel(got, d["pot"])
    ew = float(np.max(np.abs(got - d["pot"])) / np.max(np.abs(d["pot"])))
    print(f"{name} {precision}: rel L2 vs oracle {e:.3e} (max elementwise {ew:.3e}, {d['idx'].size} targets)")
    assert e < tol
    return e


TOL_P10 = {"fp64": 1e-8, "fp32": 1e-5, "bf16x3": 1e-5, "bf16x5": 1e-5, "f16x3": 1e-6,
           "fp64+m2l_fp32": 1e-6, "fp64+m2l_f16x3": 1e-6}


@pytest.mark.parametrize("precision", MODES)
def test_p10_multi_rhs_twin_vs_oracle(precision):
    name = "uniform100k_d4_p10_rhs4"
    tree, ops, qd, d = case(name)
    # the paths under test are the defaults at this order and size
    for key in ("m2l_fp64_sum_min_p", "far_fp64_min_p", "m2l_check_min_p"):
        assert K.get_tuning(key) <= 10, key
    inf = tree.info()
    assert inf.n_boxes * qd.shape[0] // 64 >= 128  # >= 128 tiles: full 160-row GEMM blocks
    check(name, precision, TOL_P10[precision])


@pytest.mark.parametrize("layout", ["default", "tiles128_pairs"])
@pytest.mark.parametrize("precision", MODES)
def test_p8_sphere_twin_vs_oracle(precision, layout):
    name = "sphere300k_nc64_p8"
    old = {k: K.get_tuning(k) for k in ("m2l_tile_cols", "m2l_pair_fill")}
    try:
        if layout == "tiles128_pairs":
            K.set_tuning("m2l_tile_cols", 128)
            K.set_tuning("m2l_pair_fill", 101)
        check(name, precision, 1e-8 if precision == "fp64" else 1e-5)
    finally:
        for k, v in old.items():
            K.set_tuning(k, v)


@pytest.mark.parametrize("precision", MODES)
def test_headline_1m_vs_oracle_sample(precision):
    check("uniform1m_d5_p6", precision, 1e-8 if precision == "fp64" else 1e-5)


def test_64_rhs_at_p10_equals_two_32_rhs_runs():
    """1M points, p = 10, 64 right-hand sides in split BF16: the M2L operand
    then spans (37,450 boxes x 64 x 512 x 2 parts) > 2^31 elements, past the
    range of 32-bit offsets.  Columns must equal two 32-column runs bitwise
    (multi-RHS columns never depend on the other columns), and FP16 split
    runs agree to its accuracy (its density scale is shared by the columns
    of one call, so the split can differ)."""
    prob = I.multi_rhs_1m(n_rhs=64)
    tree = K.Tree(prob.points, uniform_depth=prob.uniform_depth, center=prob.center, halfwidth=prob.halfwidth)
    ops = K.Operators(prob.p, device_svd=True)
    q = torch.as_tensor(prob.charges, dtype=torch.float64, device=DEV)
    for precision in ("bf16x3", "f16x3"):
        full = K.evaluate(tree, ops, q, precision=precision)
        torch.cuda.synchronize()
        full = full.cpu().numpy()
        for h in range(2):
            half = K.evaluate(tree, ops, q[32 * h:32 * (h + 1)].contiguous(), precision=precision)
            torch.cuda.synchronize()
            half = half.cpu().numpy()
            if precision == "bf16x3":
                np.testing.assert_array_equal(full[32 * h:32 * (h + 1)], half)
            else:
                assert rel(full[32 * h:32 * (h + 1)], half) < 1e-6
        print(f"64 RHS, p = 10, {precision}: columns match the 32-RHS runs")
        del full
        torch.cuda.empty_cache()
