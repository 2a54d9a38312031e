"""The allocation-free entry point (kifmm_evaluate_noalloc) through the C
ABI against kifmm_evaluate, the entry point it is a variant of: bitwise
equal potentials (same kernels, same order), on two calls in a row whose
second has the smaller input (the fixed work array keeps the first call's
values, so this also checks what must start at zero is cleared), in the
split-BF16 headline mode and in FP64, one and several right-hand sides."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2303_08394_amd import inputs as I  # noqa: E402
from paper_2303_08394_amd import kifmm as K  # noqa: E402

DEV = "cuda:0"
CUBE = dict(center=(0.5, 0.5, 0.5), halfwidth=0.5)


def noalloc(tree, ops, q, out, prec):
    L = K.lib()
    st = L.kifmm_evaluate_noalloc(tree.handle, ops.handle, C.c_void_p(q.data_ptr()), q.shape[0],
                                  C.c_void_p(out.data_ptr()), 1 if q.dtype == torch.float64 else 0,
                                  K.PRECISIONS[prec], C.c_void_p(torch.cuda.current_stream().cuda_stream))
    K._check(st)


@pytest.mark.parametrize("prec,n_rhs", [("bf16x3", 1), ("fp64", 1), ("f16x3", 3)])
def test_noalloc_equals_evaluate_twice_second_smaller(prec, n_rhs):
    ops = K.Operators(6)
    runs = []
    # the second input is smaller; three right-hand sides on smaller trees
    sizes = ((400000, 5, 71), (60000, 4, 72)) if n_rhs == 1 else ((150000, 4, 71), (40000, 3, 72))
    for n, depth, seed in sizes:
        x, q = I.uniform_cube(n, seed=seed, charge_range=(-1, 1), n_rhs=n_rhs)
        tree = K.Tree(x, uniform_depth=depth, **CUBE)
        qd = torch.as_tensor(np.atleast_2d(q), dtype=torch.float64, device=DEV).contiguous()
        want = K.evaluate(tree, ops, qd, precision=prec)  # also makes the device state resident
        torch.cuda.synchronize()
        want = want.cpu().numpy()
        out = torch.full((qd.shape[0], n), float("nan"), dtype=torch.float64, device=DEV)
        noalloc(tree, ops, qd, out, prec)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        print(f"noalloc {prec} n={n} n_rhs={n_rhs}: max |diff| {np.max(np.abs(got - want)):.3e}")
        np.testing.assert_array_equal(got, want)
        runs.append((tree, qd, want))
    # the first tree again, after the smaller one left its values in the array
    tree, qd, want = runs[0]
    out = torch.empty_like(qd)
    noalloc(tree, ops, qd, out, prec)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), want)


def test_noalloc_preconditions_and_limit():
    ops = K.Operators(4)
    x, q = I.uniform_cube(5000, seed=73)
    tree = K.Tree(x, uniform_depth=3, **CUBE)
    qd = torch.as_tensor(np.atleast_2d(q), dtype=torch.float64, device=DEV).contiguous()
    out = torch.empty_like(qd)
    with pytest.raises(K.KifmmError, match="EINVAL.*run kifmm_evaluate once"):
        noalloc(tree, ops, qd, out, "fp32")  # nothing resident yet
    K.evaluate(tree, ops, qd, precision="fp32")
    torch.cuda.synchronize()
    with pytest.raises(K.KifmmError, match="EINVAL.*run kifmm_evaluate once"):
        noalloc(tree, ops, qd, out, "fp64")  # FP64 tables not uploaded yet
    noalloc(tree, ops, qd, out, "fp32")
    torch.cuda.synchronize()
    # 1M points, two right-hand sides in plain FP64 (p = 6): ~400 MiB of work
    # buffers, more than the fixed array holds
    big_x, big_q = I.uniform_cube(1000000, seed=74, charge_range=(-1, 1), n_rhs=2)
    big = K.Tree(big_x, uniform_depth=5, **CUBE)
    ops6 = K.Operators(6)
    bq = torch.as_tensor(big_q, dtype=torch.float64, device=DEV).contiguous()
    K.evaluate(big, ops6, bq, precision="fp64")
    torch.cuda.synchronize()
    bout = torch.empty_like(bq)
    with pytest.raises(K.KifmmError, match="EUNSUPPORTED.*MiB"):
        noalloc(big, ops6, bq, bout, "fp64")
