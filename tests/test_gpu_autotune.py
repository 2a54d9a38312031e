"""The autotuner on the GPU, and the launch layouts it may pick: every layout
gives the oracle's potentials; the tile widths give them bitwise equal."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import kifmm as OK  # noqa: E402
from oracle.octree import Octree  # noqa: E402
from paper_2303_08394_amd import autotune as A  # noqa: E402
from paper_2303_08394_amd import inputs as I  # noqa: E402
from paper_2303_08394_amd import kifmm as K  # noqa: E402

CUBE = dict(center=(0.5, 0.5, 0.5), halfwidth=0.5)
DEV = "cuda:0"
TOL = {"fp64": 1e-8, "fp32": 1e-5, "bf16x3": 1e-5}
CASES = {
    "uniform20k_d3_p6": lambda: (*I.uniform_cube(20000, seed=0), 6, dict(uniform_depth=3, **CUBE)),
    "sphere12k_nc32_p6": lambda: (*I.sphere_surface(12000, seed=2), 6, dict(ncrit=32, max_depth=10)),
}
_ops, _want = {}, {}


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def setup(name):
    x, q, p, kw = CASES[name]()
    if p not in _ops:
        _ops[p] = K.Operators(p)
    if name not in _want:
        _want[name] = OK.KIFMM(Octree(x, x, **kw), p).evaluate(np.atleast_2d(q))
    return K.Tree(x, **kw), _ops[p], torch.as_tensor(q, dtype=torch.float64, device=DEV), _want[name]


def run(tree, ops, qd, precision):
    s = torch.cuda.Stream()  # graph replays, as the autotuner times them
    out = K.evaluate(tree, ops, qd, precision, stream=s)
    s.synchronize()
    return out.cpu().numpy()


def restore_defaults():
    for k, cands in A.SPACE:
        K.set_tuning(k, cands[0])


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", ["fp64", "bf16x3"])
def test_autotuned_layout_keeps_the_results(name, precision, tmp_path):
    tree, ops, qd, want = setup(name)
    print(f"autotune {name} {precision}", flush=True)
    base = run(tree, ops, qd, precision)
    cache = str(tmp_path / "tune.json")
    try:
        r = A.autotune_evaluate(tree, ops, qd, precision, cache_path=cache, steps=3, warmup=1)
        n0 = 1 + sum(len(c) - 1 for _, c in A.SPACE)
        assert len(r.trials) in (n0, n0 + 6)  # + 3 alternate re-timings when the layout moved
        assert all(t > 0 for _, t in r.trials) and r.best_ms > 0
        assert {k: K.get_tuning(k) for k, _ in A.SPACE} == r.best
        got = run(tree, ops, qd, precision)
        assert rel(got, want) < TOL[precision]
        # tile width and block shape keep every value bitwise
        same = ("m2l_tile_cols", "m2l_rows", "m2l_wide", "m2l_async")
        if all(r.best[k] == c[0] for k, c in A.SPACE if k not in same):
            np.testing.assert_array_equal(got, base)  # only bitwise-neutral knobs moved
        else:
            assert rel(got, base) < (1e-8 if precision == "fp64" else 1e-6)
        restore_defaults()
        r2 = A.autotune_evaluate(tree, ops, qd, precision, cache_path=cache)
        assert r2.from_cache and r2.best == r.best
        assert {k: K.get_tuning(k) for k, _ in A.SPACE} == r.best
    finally:
        restore_defaults()


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("width", [128, 160])
def test_wider_column_tiles_equal_64(name, precision, width):
    tree, ops, qd, want = setup(name)
    narrow = run(tree, ops, qd, precision)
    K.set_tuning("m2l_tile_cols", width)
    try:
        wide = run(tree, ops, qd, precision)
    finally:
        K.set_tuning("m2l_tile_cols", 64)
    np.testing.assert_array_equal(wide, narrow)
    assert rel(wide, want) < TOL[precision]


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_unsplit_m2l_tiles(name, precision):
    """One block per M2L tile (m2l_split 0): each output is then a single
    term, so the values differ from the two-part default only by rounding."""
    tree, ops, qd, want = setup(name)
    split = run(tree, ops, qd, precision)
    K.set_tuning("m2l_split", 0)
    try:
        whole = run(tree, ops, qd, precision)
        again = run(tree, ops, qd, precision)
    finally:
        K.set_tuning("m2l_split", 1)
    np.testing.assert_array_equal(whole, again)
    assert rel(whole, want) < TOL[precision]
    assert rel(whole, split) < (1e-8 if precision == "fp64" else 1e-6)
