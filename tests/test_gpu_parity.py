"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (relative L2 over all compared targets):
  FP64 GPU vs FP64 oracle: 1e-8.  Both sides compute their own truncated
    pseudo-inverse (Jacobi SVD vs LAPACK); with rcond = 1e-9 the operators
    agree only to ~1e-8 and the fields to ~1e-9 (measured spread between two
    correct SVD drivers), so 1e-8 is the floor a correct FP64 path can meet.
  FP32 and split-BF16 M2L vs FP64 oracle: 1e-5 (the accuracy target of the
    mixed-precision paths).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import direct, kifmm as OK  # noqa: E402
from oracle.octree import Octree  # noqa: E402
from paper_2303_08394_amd import inputs as I  # noqa: E402
from paper_2303_08394_amd import kifmm as K  # noqa: E402

CUBE = dict(center=(0.5, 0.5, 0.5), halfwidth=0.5)
TOL64, TOL32 = 1e-8, 1e-5
TOL = {"fp64": TOL64, "fp32": TOL32, "bf16x3": TOL32, "bf16x5": TOL32, "f16x3": TOL32,
       "fp64+m2l_fp32": TOL32, "fp64+m2l_f16x3": TOL32}
DEV = "cuda:0"


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


_ops = {}


def ops(p):
    if p not in _ops:
        _ops[p] = K.Operators(p)
    return _ops[p]


def gpu_eval(tree, p, q, precision, dtype=torch.float64):
    qd = torch.as_tensor(np.atleast_2d(q), dtype=dtype, device=DEV)
    out = K.evaluate(tree, ops(p), qd, precision=precision)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


_oracle_cache = {}


def oracle(name, x, q, tgt, p, **kw):
    if name not in _oracle_cache:
        t = Octree(x, tgt, **kw)
        _oracle_cache[name] = OK.KIFMM(t, p).evaluate(np.atleast_2d(q))
    return _oracle_cache[name]


CASES = {
    # name: (points, charges, targets, p, tree kwargs)
    "uniform20k_d3_p6": lambda: (*I.uniform_cube(20000, seed=0), None, 6, dict(uniform_depth=3, **CUBE)),
    "uniform3k_d3_p4_sparse": lambda: (*I.uniform_cube(3000, seed=1, charge_range=(-1, 1)), None, 4,
                                       dict(uniform_depth=3, **CUBE)),
    "sphere12k_nc32_p6": lambda: (*I.sphere_surface(12000, seed=2), None, 6, dict(ncrit=32, max_depth=10)),
    "clustered8k_nc24_p5": lambda: (*I.clustered(8000, seed=3), None, 5, dict(ncrit=24, max_depth=10, **CUBE)),
}


def _case(name):
    x, q, tgt, p, kw = CASES[name]()
    tgt = x if tgt is None else tgt
    return x, q, tgt, p, kw


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3", "bf16x5", "f16x3", "fp64+m2l_fp32",
                                       "fp64+m2l_f16x3"])
def test_parity_vs_oracle(name, precision):
    x, q, tgt, p, kw = _case(name)
    want = oracle(name, x, q, tgt, p, **kw)
    tree = K.Tree(x, tgt, **kw)
    got = gpu_eval(tree, p, q, precision)
    e = rel(got, want)
    print(f"{name} {precision} rel L2 vs oracle = {e:.3e}")
    assert e < TOL[precision]


def test_fp32_io_and_separate_targets():
    x, q = I.clustered(5000, seed=8)
    tgt = np.vstack([np.random.default_rng(8).random((3000, 3)), x[:500]])  # 500 coincide with sources
    kw = dict(ncrit=20, max_depth=9, **CUBE)
    want = OK.KIFMM(Octree(x, tgt, **kw), 5).evaluate(q)
    tree = K.Tree(x, tgt, **kw)
    got64 = gpu_eval(tree, 5, q, "fp64")
    got32 = gpu_eval(tree, 5, q, "fp32", dtype=torch.float32)
    assert rel(got64, want) < TOL64
    assert rel(got32, want) < TOL32


def test_multi_rhs_equals_single_columns():
    x, _ = I.uniform_cube(6000, seed=9)
    qm = np.random.default_rng(9).uniform(-1, 1, (3, 6000))
    tree = K.Tree(x, uniform_depth=3, **CUBE)
    for prec in ("fp32", "fp64"):
        m = gpu_eval(tree, 5, qm, prec)
        for r in range(3):
            s = gpu_eval(tree, 5, qm[r], prec)
            np.testing.assert_array_equal(m[r], s[0])


def test_batch_equals_individual_runs():
    probs = [I.uniform_cube(n, seed=10 + n) for n in (2000, 5000, 3500)]
    probs.append(I.clustered(4000, seed=14))
    trees = [K.Tree(x, ncrit=32, max_depth=10, **CUBE) for x, _ in probs]
    qs = [torch.as_tensor(q[0], dtype=torch.float64, device=DEV) for _, q in probs]
    outs = K.evaluate_batch(trees, ops(5), qs, precision="fp32")
    torch.cuda.synchronize()
    for t, (x, q), o in zip(trees, probs, outs):
        single = gpu_eval(t, 5, q, "fp32")[0]
        np.testing.assert_array_equal(o.cpu().numpy(), single)


def test_deterministic():
    x, q = I.uniform_cube(8000, seed=15, charge_range=(-1, 1))
    tree = K.Tree(x, uniform_depth=3, **CUBE)
    a = gpu_eval(tree, 6, q, "fp32")
    b = gpu_eval(tree, 6, q, "fp32")
    np.testing.assert_array_equal(a, b)


def test_degenerate_inputs():
    # one point: no other charge, the potential is exactly zero
    t = K.Tree(np.array([[0.3, 0.3, 0.3]]), ncrit=4, max_depth=5)
    assert gpu_eval(t, 4, np.array([2.0]), "fp32")[0, 0] == 0.0
    # two points: closed form
    x = np.array([[0.1, 0.2, 0.3], [0.7, 0.1, 0.4]])
    t = K.Tree(x, ncrit=1, max_depth=5)
    got = gpu_eval(t, 4, np.array([1.0, 2.0]), "fp64")[0]
    r = np.linalg.norm(x[0] - x[1])
    np.testing.assert_allclose(got, [2 / (4 * np.pi * r), 1 / (4 * np.pi * r)], rtol=1e-12)
    # all points on a plane, and repeated points
    rng = np.random.default_rng(16)
    x = np.c_[rng.random((3000, 2)), np.full(3000, 0.5)]
    x[100:110] = x[0]
    q = rng.random(3000)
    kw = dict(ncrit=16, max_depth=10, **CUBE)
    want = OK.KIFMM(Octree(x, x, **kw), 4).evaluate(q)
    assert rel(gpu_eval(K.Tree(x, **kw), 4, q, "fp64")[0], want) < TOL64
    # zero charges
    assert np.all(gpu_eval(K.Tree(x, **kw), 4, 0 * q, "fp32") == 0)


def test_evaluate_simple_matches_direct():
    x, q = I.sphere_surface(4000, seed=17)
    got = K.evaluate_simple(x, q[0], x, 6)
    assert rel(got, direct.direct(x, q[0], x)) < 1e-5


@pytest.mark.parametrize("precision", ["fp32", "f16x3", "fp64+m2l_f16x3"])
def test_check_form_m2l(precision):
    """M2L on upward check potentials with operators folded with UC2E (the
    high-order form), forced at low order, against the oracle."""
    name = "uniform20k_d3_p6"
    x, q, tgt, p, kw = _case(name)
    want = oracle(name, x, q, tgt, p, **kw)
    K.set_tuning("m2l_check_min_p", 2)
    try:
        tree = K.Tree(x, tgt, **kw)
        got = gpu_eval(tree, p, q, precision)
    finally:
        K.set_tuning("m2l_check_min_p", 10)
        _ops.clear()
    e = rel(got, want)
    print(f"check-form {precision} rel L2 vs oracle = {e:.3e}")
    assert e < TOL32


def test_graph_replays_match_eager():
    """Captured evaluations replayed several times, with eager work and
    synchronisation between the replays, equal the eager result bitwise."""
    x, _ = I.uniform_cube(8000, seed=31)
    rng = np.random.default_rng(31)
    charges = [rng.uniform(-1, 1, 8000) for _ in range(4)]
    tree = K.Tree(x, uniform_depth=3, **CUBE)
    s = torch.cuda.Stream()
    qbuf = torch.empty(8000, dtype=torch.float64, device=DEV)
    obuf = torch.empty((1, 8000), dtype=torch.float64, device=DEV)
    for prec in ("f16x3", "fp64"):
        K.set_tuning("graph", 0)
        eager = []
        with torch.cuda.stream(s):
            for c in charges:
                qbuf.copy_(torch.as_tensor(c, device=DEV))
                K.evaluate(tree, ops(5), qbuf, precision=prec, out=obuf)
                s.synchronize()
                eager.append(obuf.cpu().numpy().copy())
        K.set_tuning("graph", 1)
        try:
            with torch.cuda.stream(s):
                for rep in range(2):
                    for c, want in zip(charges, eager):
                        qbuf.copy_(torch.as_tensor(c, device=DEV))
                        K.evaluate(tree, ops(5), qbuf, precision=prec, out=obuf)
                        s.synchronize()
                        junk = torch.randn(1000, device=DEV).sum()  # eager work between replays
                        torch.cuda.synchronize()
                        np.testing.assert_array_equal(obuf.cpu().numpy(), want)
        finally:
            K.set_tuning("graph", 1)


def test_new_operator_set_is_captured_anew():
    """An evaluation with a new operator set of the same order, made after
    the old one was destroyed (its tables freed, its address free for
    reuse), captures a new graph instead of replaying one that points at the
    freed tables; results equal the first evaluation bitwise."""
    x, q = I.uniform_cube(6000, seed=32, charge_range=(-1, 1))
    tree = K.Tree(x, uniform_depth=3, **CUBE)
    s = torch.cuda.Stream()
    qd = torch.as_tensor(np.atleast_2d(q), dtype=torch.float64, device=DEV)
    out = torch.empty_like(qd)
    with torch.cuda.stream(s):
        a = K.Operators(4)
        K.evaluate(tree, a, qd, precision="fp32", out=out)
        s.synchronize()
        first = out.cpu().numpy().copy()
        n0 = K.graph_captures()
        K.evaluate(tree, a, qd, precision="fp32", out=out)  # replay, no capture
        s.synchronize()
        assert K.graph_captures() == n0
        del a
        import gc
        gc.collect()
        for _ in range(3):
            b = K.Operators(4)
            out.zero_()
            K.evaluate(tree, b, qd, precision="fp32", out=out)
            s.synchronize()
            assert K.graph_captures() == n0 + 1
            np.testing.assert_array_equal(out.cpu().numpy(), first)
            del b
            gc.collect()
            n0 += 1


def test_batch_graph_replays_match_eager():
    probs = [I.clustered(n, seed=40 + n) for n in (3000, 5000, 2000)]
    trees = [K.Tree(xx, ncrit=32, max_depth=10, **CUBE) for xx, _ in probs]
    qs = [torch.as_tensor(q[0], dtype=torch.float64, device=DEV) for _, q in probs]
    s = torch.cuda.Stream()
    K.set_tuning("graph", 0)
    with torch.cuda.stream(s):
        eager = [o.cpu().numpy() for o in K.evaluate_batch(trees, ops(5), qs, precision="fp32")]
    K.set_tuning("graph", 1)
    outs = [torch.empty_like(q) for q in qs]
    with torch.cuda.stream(s):
        for rep in range(3):
            K.evaluate_batch(trees, ops(5), qs, precision="fp32", outs=outs)
            s.synchronize()
            for o, w in zip(outs, eager):
                np.testing.assert_array_equal(o.cpu().numpy(), w)


@pytest.mark.parametrize("precision", ["bf16x3", "f16x3", "fp32"])
def test_wide_m2l_tiles_equal_narrow(precision):
    """192-column M2L tiles (768-thread blocks) give the same values, bitwise,
    as 64-column tiles: every box's M2L is the sum of its two parity parts,
    each accumulated over its offsets in the same order whatever the tile."""
    name = "sphere12k_nc32_p6"
    x, q, tgt, p, kw = _case(name)
    tree = K.Tree(x, tgt, **kw)
    narrow = gpu_eval(tree, p, q, precision)
    K.set_tuning("m2l_tile_cols", 192)
    try:
        wide = gpu_eval(tree, p, q, precision)  # the plans are rebuilt for the new width
    finally:
        K.set_tuning("m2l_tile_cols", 64)
    np.testing.assert_array_equal(wide, narrow)
    want = oracle(name, x, q, tgt, p, **kw)
    assert rel(wide, want) < TOL32


@pytest.mark.parametrize("case", [("uniform20k_d3_p6", 1), ("uniform20k_d3_p6", 2), ("uniform20k_d3_p6", 3),
                                  ("uniform3k_d3_p4_sparse", 1), ("clustered8k_nc24_p5", 1), ("p8", 1)])
@pytest.mark.parametrize("precision", ["bf16x3", "f16x3", "fp64+m2l_f16x3"])
def test_wide_tile_kernel_equals_gemm_kernel(case, precision):
    """The wide-tile split M2L kernel (128-column plans) gives gemm_kernel's
    results bitwise: the same plans, products and per-column summation order.
    Cases cover 1, 2 and 3 right-hand sides (tiles of 128, 64 and 42 boxes:
    ragged columns), operators shorter than the 160-row block (p = 4, 5),
    two row blocks (p = 8), adaptive trees, and FP64 outputs."""
    name, n_rhs = case
    if name == "p8":
        x, q = I.uniform_cube(12000, seed=33, charge_range=(-1, 1))
        tgt, p, kw = None, 8, dict(uniform_depth=3, **CUBE)
    else:
        x, q, tgt, p, kw = CASES[name]()
    tree = K.Tree(x, tgt, **kw)
    qm = np.vstack([np.atleast_2d(q)] + [np.random.default_rng(40 + r).uniform(-1, 1, (1, len(x)))
                                         for r in range(n_rhs - 1)])
    K.set_tuning("m2l_tile_cols", 128)
    K.set_tuning("m2l_async", 0)
    try:
        K.set_tuning("m2l_wide", 0)
        ref = gpu_eval(tree, p, qm, precision)
        K.set_tuning("m2l_wide", 1)
        got = gpu_eval(tree, p, qm, precision)
    finally:
        K.set_tuning("m2l_tile_cols", 64)
        K.set_tuning("m2l_wide", 0)
        K.set_tuning("m2l_async", 1)
    np.testing.assert_array_equal(got, ref)
    narrow = gpu_eval(tree, p, qm, precision)
    np.testing.assert_array_equal(got, narrow)


@pytest.mark.parametrize("case", [("uniform20k_d3_p6", 1), ("uniform20k_d3_p6", 2), ("uniform20k_d3_p6", 3),
                                  ("uniform3k_d3_p4_sparse", 1), ("clustered8k_nc24_p5", 1), ("p8", 1),
                                  ("p7", 2)])
@pytest.mark.parametrize("precision", ["bf16x3", "f16x3", "fp64+m2l_f16x3"])
@pytest.mark.parametrize("width", [64, 96, 128, 160])
def test_async_staging_kernel_equals_gemm_kernel(case, precision, width):
    """The split M2L kernel that stages chunks straight from global memory into
    LDS (plans of 64, 96, 128 and 160 columns) gives gemm_kernel's results bitwise:
    the same plans, products and per-column summation order.  Cases: 1, 2 and 3
    right-hand sides (ragged columns: tiles of 21, 42 or 53 boxes), operators
    shorter than the block (p = 4), 128-row blocks (p = 5, 7), two row blocks
    (p = 8), adaptive trees, FP64 outputs."""
    name, n_rhs = case
    if name in ("p8", "p7"):
        x, q = I.uniform_cube(12000, seed=33, charge_range=(-1, 1))
        tgt, p, kw = None, int(name[1]), dict(uniform_depth=3, **CUBE)
    else:
        x, q, tgt, p, kw = CASES[name]()
    tree = K.Tree(x, tgt, **kw)
    qm = np.vstack([np.atleast_2d(q)] + [np.random.default_rng(40 + r).uniform(-1, 1, (1, len(x)))
                                         for r in range(n_rhs - 1)])
    K.set_tuning("m2l_tile_cols", width)
    try:
        K.set_tuning("m2l_async", 0)
        ref = gpu_eval(tree, p, qm, precision)
        K.set_tuning("m2l_async", 1)
        got = gpu_eval(tree, p, qm, precision)
    finally:
        K.set_tuning("m2l_async", 1)
        K.set_tuning("m2l_tile_cols", 64)
    np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("case", [("uniform20k_d3_p6", 1), ("uniform20k_d3_p6", 3), ("clustered8k_nc24_p5", 1),
                                  ("p8", 2), ("p10", 1)])
@pytest.mark.parametrize("precision", ["bf16x3", "f16x3", "fp64+m2l_f16x3"])
@pytest.mark.parametrize("width", [64, 96])
def test_async_staging_kernel_with_fp64_sums(case, precision, width):
    """With FP64 sums after every operator step (the default from p = 10; here
    forced from p = 2 on), M2L tiles of 64 and 96 columns staged straight into
    LDS give gemm_kernel's results bitwise: the same per-step FP32 sums, moved
    into FP64 at the same points (96 columns with 128-row blocks only; with
    160-row blocks such tiles run gemm_kernel).  Cases: 1, 2, 3 right-hand
    sides, 128-row blocks (p = 5, 10), two row blocks (p = 8), an adaptive
    tree."""
    name, n_rhs = case
    if name in ("p8", "p10"):
        x, q = I.uniform_cube(12000 if name == "p8" else 6000, seed=36, charge_range=(-1, 1))
        tgt, p, kw = None, int(name[1:]), dict(uniform_depth=3, **CUBE)
    else:
        x, q, tgt, p, kw = CASES[name]()
    tree = K.Tree(x, tgt, **kw)
    qm = np.vstack([np.atleast_2d(q)] + [np.random.default_rng(50 + r).uniform(-1, 1, (1, len(x)))
                                         for r in range(n_rhs - 1)])
    K.set_tuning("m2l_fp64_sum_min_p", 2)
    K.set_tuning("m2l_tile_cols", width)
    try:
        K.set_tuning("m2l_async", 0)
        ref = gpu_eval(tree, p, qm, precision)
        K.set_tuning("m2l_async", 1)
        got = gpu_eval(tree, p, qm, precision)
    finally:
        K.set_tuning("m2l_async", 1)
        K.set_tuning("m2l_fp64_sum_min_p", 10)
        K.set_tuning("m2l_tile_cols", 64)
    np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("name", ["sphere12k_nc32_p6", "uniform3k_d3_p4_sparse", "p8"])
@pytest.mark.parametrize("precision", ["bf16x3", "f16x3"])
@pytest.mark.parametrize("width", [64, 128, 160])
def test_async_staging_kernel_on_pair_tiles(name, precision, width):
    """M2L run pair by pair: the pair tiles (one offset each, products stored
    to the pair buffer, not added) staged straight into LDS give gemm_kernel's
    pair products, hence the same potentials bitwise.  Operators of one and
    two row blocks (p = 4, 6; p = 8), ragged last tiles."""
    if name == "p8":
        x, q = I.uniform_cube(12000, seed=35, charge_range=(-1, 1))
        tgt, p, kw = None, 8, dict(uniform_depth=3, **CUBE)
    else:
        x, q, tgt, p, kw = CASES[name]()
    tree = K.Tree(x, tgt, **kw)
    K.set_tuning("m2l_tile_cols", width)
    K.set_tuning("m2l_pair_fill", 101)  # every problem pair by pair
    try:
        K.set_tuning("m2l_async", 0)
        ref = gpu_eval(tree, p, q, precision)
        K.set_tuning("m2l_async", 1)
        got = gpu_eval(tree, p, q, precision)
    finally:
        K.set_tuning("m2l_async", 1)
        K.set_tuning("m2l_pair_fill", 40)
        K.set_tuning("m2l_tile_cols", 64)
    np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("p", [5, 6, 7])
@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "f16x3", "fp64"])
def test_m2l_block_rows_do_not_change_results(p, precision):
    """M2L blocks of 160 or 128 operator rows (m2l_rows) give the same
    potentials bitwise: rows are independent outputs.  p = 5 and 7 (ld 128,
    224) default to 128-row blocks, p = 6 to 160."""
    x, q = I.uniform_cube(6000, seed=34, charge_range=(-1, 1))
    tree = K.Tree(x, uniform_depth=3, **CUBE)
    outs = []
    try:
        for rows in (0, 160, 128):
            K.set_tuning("m2l_rows", rows)
            outs.append(gpu_eval(tree, p, q, precision))
    finally:
        K.set_tuning("m2l_rows", 0)
    np.testing.assert_array_equal(outs[1], outs[0])
    np.testing.assert_array_equal(outs[2], outs[0])


@pytest.mark.parametrize("fork", [0, 1, 2, 3])
@pytest.mark.parametrize("precision", ["fp64", "bf16x3"])
def test_near_field_schedules(fork, precision):
    """Every place of the near field in the schedule gives the oracle's
    potentials: the default (near and far field summed by one kernel at the
    end) and the near field as its own kernel on a second stream, forked after
    the gather, after P2M, before or after M2L.  The forked schedules differ
    from the default only in the rounding of the near + far sum; among
    themselves they only move the same kernels between streams, so they agree
    bitwise."""
    name = "sphere12k_nc32_p6"
    x, q, tgt, p, kw = _case(name)
    tree = K.Tree(x, tgt, **kw)
    merged = gpu_eval(tree, p, q, precision)
    K.set_tuning("near_fork", fork)
    try:
        got = gpu_eval(tree, p, q, precision)
        K.set_tuning("near_fork", 0)
        first = gpu_eval(tree, p, q, precision)
    finally:
        K.set_tuning("near_fork", 4)
    np.testing.assert_array_equal(got, first)
    assert rel(got, merged) < (1e-13 if precision == "fp64" else 1e-6)
    want = oracle(name, x, q, tgt, p, **kw)
    assert rel(got, want) < TOL[precision]


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3", "f16x3"])
def test_m2l_pair_scheme(name, precision):
    """M2L run pair by pair (one product per V-list pair, then each target's
    sum in offset order) gives the oracle's potentials, and agrees with the
    gathered tiles up to the rounding of the sums.  (In FP64 the rounding
    differences of the check potentials pass through the check-to-equivalent
    solves, whose pseudo-inverse keeps singular values down to 1e-9 of the
    largest: measured ~5e-10 on the potentials, bounded by TOL64.)"""
    x, q, tgt, p, kw = _case(name)
    tree = K.Tree(x, tgt, **kw)
    K.set_tuning("m2l_pair_fill", 101)  # every problem pair by pair
    try:
        pairs = gpu_eval(tree, p, q, precision)
        K.set_tuning("m2l_pair_fill", 0)  # every problem in gathered tiles
        tiles = gpu_eval(tree, p, q, precision)
    finally:
        K.set_tuning("m2l_pair_fill", 40)
    want = oracle(name, x, q, tgt, p, **kw)
    assert rel(pairs, want) < TOL[precision]
    assert rel(pairs, tiles) < (TOL64 if precision == "fp64" else 1e-6)


def test_batch_mixed_m2l_schemes_equal_individual_runs():
    """A batch whose problems take different M2L schemes reproduces each
    problem's single run bitwise (at a 20% threshold the sphere's tiles, ~7%
    full, run pair by pair and the cube's, ~29% full, as gathered tiles); so
    do multi-RHS columns run pair by pair."""
    xs, qs0 = I.sphere_surface(6000, seed=21)
    xc, qc0 = I.uniform_cube(5000, seed=22)
    trees = [K.Tree(xs, ncrit=32, max_depth=10), K.Tree(xc, uniform_depth=3, **CUBE)]
    K.set_tuning("m2l_pair_fill", 20)
    try:
        for prec in ("fp32", "bf16x3"):
            qs = [torch.as_tensor(q[0], dtype=torch.float64, device=DEV) for q in (qs0, qc0)]
            outs = K.evaluate_batch(trees, ops(5), qs, precision=prec)
            torch.cuda.synchronize()
            for t, q, o in zip(trees, (qs0, qc0), outs):
                single = gpu_eval(t, 5, q, prec)[0]
                np.testing.assert_array_equal(o.cpu().numpy(), single)
    finally:
        K.set_tuning("m2l_pair_fill", 40)
    qm = np.random.default_rng(23).uniform(-1, 1, (3, 6000))
    K.set_tuning("m2l_pair_fill", 101)
    try:
        m = gpu_eval(trees[0], 5, qm, "fp32")
        for r in range(3):
            np.testing.assert_array_equal(m[r], gpu_eval(trees[0], 5, qm[r], "fp32")[0])
    finally:
        K.set_tuning("m2l_pair_fill", 40)


@pytest.mark.parametrize("precision", ["bf16x3", "f16x3", "fp32"])
def test_zero_and_scaled_charges(precision):
    """Zero charges give zero potentials; scaling the charges by 2^-66 or 2^66
    (about 1e-20 and 1e20) scales the potentials exactly: every rounding of
    the path commutes with a power of two while nothing leaves the normal
    range (the FP16 split rescales the densities by a power of two taken from
    their largest magnitude, the BF16 split shares FP32's exponent range)."""
    x, q = I.uniform_cube(5000, seed=50, charge_range=(-1, 1))
    tree = K.Tree(x, uniform_depth=3, **CUBE)
    assert np.all(gpu_eval(tree, 5, 0 * q, precision) == 0)
    base = gpu_eval(tree, 5, q, precision)
    for s in (2.0 ** -66, 2.0 ** 66):
        got = gpu_eval(tree, 5, s * q, precision)
        np.testing.assert_array_equal(got / s, base)
