"""Out-of-memory paths on the GPU, forced with the allocation-failure hook
(kifmm_debug_fail_allocations): every allocation point on the first
evaluation of a tree (plans, device forest, operator tables, work buffers,
split operand, pair buffer), of the device tree build and of the point
re-sort fails in turn with ENOMEM; after each failure the same call without
the hook gives the result of a run that never failed, bitwise."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2303_08394_amd import inputs as I  # noqa: E402
from paper_2303_08394_amd import kifmm as K  # noqa: E402

DEV = "cuda:0"
CUBE = dict(center=(0.5, 0.5, 0.5), halfwidth=0.5)


def _fail_each_point(call, limit=3000):
    """Arms the hook at 0, 1, 2, ... until `call` succeeds with it armed;
    returns the number of allocation points it passed.  Where the call keeps
    what it allocated before a failure, each round moves the failure one
    allocation point further."""
    for k in range(limit):
        K.fail_allocations_after(k)
        try:
            call()
        except K.KifmmError as e:
            assert "ENOMEM" in str(e) and "injected" in str(e), str(e)
            continue
        finally:
            K.fail_allocations_after(-1)
        return k
    raise AssertionError("more allocation points than expected")


@pytest.mark.parametrize("precision", ["bf16x3", "fp64"])
def test_first_evaluation_survives_each_failed_allocation(precision):
    x, q = I.sphere_surface(20000, seed=95)  # adaptive, with a pair-by-pair M2L
    kw = dict(ncrit=32, max_depth=12)
    qd = torch.as_tensor(np.atleast_2d(q), dtype=torch.float64, device=DEV)
    ref = K.evaluate(K.Tree(x, **kw), K.Operators(5), qd, precision=precision)
    torch.cuda.synchronize()
    ref = ref.cpu().numpy()
    # one tree and one operator set whose first evaluation fails at every
    # allocation point in turn (plans, device forest, tables, work buffers)
    tree, ops = K.Tree(x, **kw), K.Operators(5)
    state = {}

    def first_eval():
        out = K.evaluate(tree, ops, qd, precision=precision)
        torch.cuda.synchronize()
        state["out"] = out.cpu().numpy()

    n = _fail_each_point(first_eval)
    assert n >= 1
    np.testing.assert_array_equal(state["out"], ref)
    # a fresh pair whose first evaluation failed once, part way
    tree2, ops2 = K.Tree(x, **kw), K.Operators(5)
    K.fail_allocations_after(7)
    with pytest.raises(K.KifmmError, match="ENOMEM"):
        K.evaluate(tree2, ops2, qd, precision=precision)
    K.fail_allocations_after(-1)
    out = K.evaluate(tree2, ops2, qd, precision=precision)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), ref)


def test_device_tree_build_and_update_survive_each_failed_allocation():
    x, q = I.clustered(15000, seed=96)
    kw = dict(ncrit=24, max_depth=10, **CUBE)
    xd = torch.as_tensor(x, dtype=torch.float64, device=DEV)
    want = K.Tree(x, **kw)
    got = {}

    def build():
        got["t"] = K.Tree.on_device(xd, **kw)

    assert _fail_each_point(build) >= 5
    assert got["t"].info().n_boxes == want.info().n_boxes
    np.testing.assert_array_equal(got["t"].list(K.LIST_V)[1], want.list(K.LIST_V)[1])
    # the point re-sort of a uniform tree
    xu, qu = I.uniform_cube(20000, seed=97)
    tree = K.Tree(xu, uniform_depth=3, **CUBE)
    before = K.evaluate(tree, K.Operators(4), torch.as_tensor(qu, dtype=torch.float64, device=DEV))
    torch.cuda.synchronize()
    before = before.cpu().numpy()
    xud = torch.as_tensor(xu, dtype=torch.float64, device=DEV)
    _fail_each_point(lambda: tree.update_points(xud))
    after = K.evaluate(tree, K.Operators(4), torch.as_tensor(qu, dtype=torch.float64, device=DEV))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(after.cpu().numpy(), before)
