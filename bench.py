#!/usr/bin/env python3
"""Benchmark of the KIFMM evaluation on one MI355X.

A step is one full evaluation (gather, near field, P2M, M2M, UC2E, M2L,
P2L, L2L, DC2E, far field (L2P + M2P), scatter) of the 1M-point uniform-cube
workload (p = 6, uniform depth 5, charges in [-1, 1)) with the tree, the
operators and the charges already resident in HBM.  The headline is the
fastest mixed-precision path within the 1e-5 bound (FP32 bulk arithmetic,
M2L as three split-BF16 products, FP64 check-to-equivalent solves and FP64
per-target sums); the plain FP64 path runs on the same tree as the
comparison leg, and its result is the reference of the reported error.
Before timing, the launch layout (M2L tile width and split, pair-scheme
threshold, near-field schedule) is searched on the workload itself by
paper_2303_08394_amd.autotune and the fastest left in force (--no-autotune
keeps the library defaults); the line reports the layout that was timed.

Prints one JSON line.  --gpus N with N > 1 exits: the evaluation runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_MFMA = 157.3e12   # dense FP32 matrix FLOP/s
PEAK_FP64_MFMA = 78.6e12
PEAK_BF16_MFMA = 2.5e15     # dense BF16 / FP16 matrix FLOP/s
PEAK_HBM = 8.0e12
# The particle kernels are bound by plain FP32 VALU issue: 256 CUs x 4 SIMDs x
# 16 lanes x 2.4 GHz = 3.93e13 lane-instructions/s.  The compiled source loop
# of the leaf kernel issues 37 VALU instructions per four pairs that need no
# coincidence test (per pair 3 sub, mul + 2 fma for r^2, rsqrt, fma for the
# sum; plus the loop's own index and bound updates), counted one issue slot
# each: the rocprofv3 counters show this kernel issuing slightly more than one
# VALU instruction per 4 clocks per SIMD, so the reciprocal square root does
# not cost the main pipe more than one slot.  9.25 slots per pair.
VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9
SLOTS_PER_PAIR = 37.0 / 4.0
PEAK_PAIRS = VALU_LANE_OPS / SLOTS_PER_PAIR
# A second, tighter bound: the minimal pair itself, 8 issue slots (3 sub,
# mul + 2 fma for r^2, rsqrt, fma for the sum), no loop overhead.
PEAK_PAIRS_MIN_OPS = VALU_LANE_OPS / 8.0


def _work_counts(tree, pn):
    """(V-list pairs, near-field pair interactions, leaf far-field pairs)."""
    from paper_2303_08394_amd import kifmm as K
    bx = tree.boxes()
    nt = bx["tgt_range"][:, 1] - bx["tgt_range"][:, 0]
    ns = bx["src_range"][:, 1] - bx["src_range"][:, 0]
    uoff, uitems = tree.list(K.LIST_U)
    woff, _ = tree.list(K.LIST_W)
    per_box_src = np.zeros(len(nt), np.int64)
    nz = np.nonzero(np.diff(uoff))[0]
    if len(uitems):
        per_box_src[nz] = np.add.reduceat(ns[uitems], uoff[nz])
    leaves = bx["is_leaf"] == 1
    near = int((nt * per_box_src)[leaves].sum())
    far = int(nt[leaves & (bx["level"] >= 2)].sum()) * pn + int((nt * np.diff(woff))[leaves].sum()) * pn
    return int(tree.info().n_v), near, far


def _translation_counts(tree):
    """Box columns of the equivalent-density solves and translations: (UC2E,
    DC2E, M2M, L2L) = (boxes of levels >= 2 with sources, with targets,
    boxes of levels >= 3 with sources, with targets)."""
    bx = tree.boxes()
    lev = bx["level"]
    ns = bx["src_range"][:, 1] - bx["src_range"][:, 0]
    nt = bx["tgt_range"][:, 1] - bx["tgt_range"][:, 0]
    return (int(((lev >= 2) & (ns > 0)).sum()), int(((lev >= 2) & (nt > 0)).sum()),
            int(((lev >= 3) & (ns > 0)).sum()), int(((lev >= 3) & (nt > 0)).sum()))


def _kernel_source_sha() -> str:
    import hashlib
    p = os.path.join(ROOT, "paper_2303_08394_amd", "csrc", "evaluate.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def _profile_value(name: str, key: str):
    """A value from a committed rocprofv3 PMC summary under profiles/, or None
    when the summary is missing, lacks the key, or was taken on another
    version of the kernel source."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip().split()[0] if v.strip() else ""
    if kv.get("evaluate_hip_sha256_16") != _kernel_source_sha():
        return None
    return float(kv[key]) if key in kv else None


def _measured_traffic(key: str):
    """HBM bytes per M2L launch (FETCH_SIZE + WRITE_SIZE, scaled by the
    copy-kernel calibration); key: the precision, with _tileN for M2L tiles
    of N columns other than 64."""
    return _profile_value("m2l_traffic_uniform1m_p6.txt", f"traffic_bytes_{key}")


# Headline mixed mode: FP32 bulk, FP64 solves and per-target sums, M2L as
# three split-BF16 products with FP32 accumulation, the fastest mode within the
# 1e-5 bound at 1M points (4.6e-6 vs plain FP64; the split-FP16 mode is 4x more
# accurate and ~4% slower).  The multi-RHS workload, bound 1e-6, uses split FP16.
DEFAULT_PRECISION = {"uniform_1m": "bf16x3", "plain_20k": "fp64", "sphere_4m": "bf16x3",
                     "batch_64": "fp32", "multi_rhs_1m": "f16x3", "paper_sphere_1m": "f16x3",
                     "screened_1m": "bf16x3"}
# the screened (Yukawa) kernel's workload: the 1M cube with kappa = 10 / the domain size
SCREENED_KAPPA = 10.0


def _problems(args):
    """The workload's problems (one, or the 64 of the batch)."""
    from paper_2303_08394_amd import inputs as I
    if args.config == "uniform_1m":
        return [I.uniform_1m()]
    if args.config == "plain_20k":
        return [I.plain_fp64_20k()]
    if args.config == "sphere_4m":
        return [I.sphere_4m()]
    if args.config == "batch_64":
        return [I.batch_problem(k) for k in range(64)]
    if args.config == "multi_rhs_1m":
        return [I.multi_rhs_1m()]
    if args.config == "paper_sphere_1m":
        return [I.paper_sphere_1m()]
    if args.config == "screened_1m":
        return [I.uniform_1m()]
    raise SystemExit(f"unknown config {args.config}")


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline():
    """The FP64 oracle as it stands, on a bounded sample of the same recipe:
    N = 125,000 uniform-cube points with uniform depth 4 (the same ~30.5
    points per leaf and p = 6 as the 1M workload), timed twice on this host:
    with one BLAS thread and with BLAS threads on every core the process may
    use (len(os.sched_getaffinity(0))); its BLAS calls are small per-box
    products, so more threads do not help it.  `value` is the faster of the
    two, `cores` the threads that run used.  Beside it, the direct sum of
    Eq. (1) (the O(N^2) oracle) timed on all targets of the 20k workload."""
    from threadpoolctl import threadpool_limits

    from oracle import direct
    from oracle import kifmm as OK
    from oracle.octree import Octree
    from paper_2303_08394_amd import inputs as I
    n = 125_000
    avail = len(os.sched_getaffinity(0))
    x, q = I.uniform_cube(n, seed=0, charge_range=(-1.0, 1.0))
    t0 = time.perf_counter()
    tree = Octree(x, x, uniform_depth=4, center=I.UNIT_CUBE_CENTER, halfwidth=I.UNIT_CUBE_HALFWIDTH)
    fm = OK.KIFMM(tree, 6)
    fm.evaluate(q[0], sample=np.arange(1))  # forms the operators (setup, not timed)
    t_setup = time.perf_counter() - t0
    runs = {}
    for threads, reps in ((1, 1), (avail, 1)):
        with threadpool_limits(limits=threads):
            ta = time.perf_counter()
            for _ in range(reps):
                fm.evaluate(q[0])
            runs[threads] = (time.perf_counter() - ta) / reps
    best = min(runs, key=runs.get)
    c1 = I.plain_fp64_20k()
    ta = time.perf_counter()
    direct.direct(c1.points, c1.charges[0], c1.points)
    t_o1 = time.perf_counter() - ta
    return {"value": n / runs[best] / 1e6, "unit": "Mpoints/s", "cores": best, "kind": "oracle",
            "sample": f"FP64 oracle evaluate, N={n} uniform cube, depth 4 (30.5 pts/leaf), p=6; "
                      f"{runs[1]:.1f} s on 1 BLAS thread, {runs[avail]:.1f} s on {avail} "
                      f"(setup {t_setup:.1f} s, not counted)",
            "host_cores_available": avail, "cpu_model": _cpu_model(),
            "evaluate_s_by_threads": {str(k): v for k, v in runs.items()},
            "direct_sum_20k_all_targets_s": t_o1,
            "direct_sum_20k_Mpairs_per_s": c1.n * (c1.n - 1) / t_o1 / 1e6}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="uniform_1m",
                    choices=["uniform_1m", "plain_20k", "sphere_4m", "batch_64", "multi_rhs_1m", "screened_1m",
                             "paper_sphere_1m"])
    ap.add_argument("--precision", default=None, choices=["fp32", "bf16x3", "bf16x5", "f16x3", "fp64", "fp64+m2l_fp32", "fp64+m2l_f16x3"])
    ap.add_argument("--no-fp64-leg", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="time eager launches instead of graph replays")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-gradient", action="store_true", help="skip the potential + gradient leg")
    ap.add_argument("--direct-sample", type=int, default=200)
    ap.add_argument("--m2l-tile", type=int, default=0, help="M2L output columns per block (64/128/192)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the launch-layout search (paper_2303_08394_amd.autotune) before timing")
    ap.add_argument("--m2l-pair-fill", type=int, default=-1,
                    help="problems whose M2L tiles are less full than this (percent) run M2L pair by pair")
    ap.add_argument("--near-fork", type=int, default=-1,
                    help="fork the near field after the gather (0) or before M2L (1)")
    ap.add_argument("--tune", action="append", default=[], metavar="KEY=VALUE",
                    help="set a tuning knob (kifmm_set_tuning) before anything runs; repeatable")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="first run one plain device copy of this many MiB (calibrates HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the evaluation runs on one GPU; --gpus {args.gpus} is not supported "
              "(a multi-GPU partition is designed, not implemented)", file=sys.stderr)
        return 2

    import torch

    from oracle import direct
    from paper_2303_08394_amd import inputs as I
    from paper_2303_08394_amd import kifmm as K

    for kv in args.tune:
        key, _, val = kv.partition("=")
        K.set_tuning(key, int(val))
    if args.m2l_tile:
        K.set_tuning("m2l_tile_cols", args.m2l_tile)
    if args.m2l_pair_fill >= 0:
        K.set_tuning("m2l_pair_fill", args.m2l_pair_fill)
    if args.near_fork >= 0:
        K.set_tuning("near_fork", args.near_fork)
    if args.copy_probe:
        # plain device copy of known size, read from HBM: the source is pushed
        # out of L2 and the 256 MB Infinity Cache by a 1 GiB fill first
        src = torch.ones(args.copy_probe * (1 << 20) // 4, dtype=torch.float32, device="cuda:0")
        flush = torch.empty(1 << 28, dtype=torch.float32, device="cuda:0")
        flush.fill_(2.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst, flush
    probs = _problems(args)
    batch = len(probs) > 1
    prob = probs[0]
    t0 = time.perf_counter()
    trees = [K.Tree(p.points, uniform_depth=p.uniform_depth, ncrit=p.ncrit, max_depth=p.max_depth,
                    center=p.center, halfwidth=p.halfwidth) for p in probs]
    t_tree = time.perf_counter() - t0
    t0 = time.perf_counter()
    # the pseudo-inverses on the GPU from p = 8 on (their host SVD dominates
    # there: 7 s at p = 10); below, the host is as fast
    ops_on_gpu = prob.p >= 8
    kappa = SCREENED_KAPPA if args.config == "screened_1m" else 0.0
    if kappa:
        ops = K.Operators.screened(prob.p, kappa, trees[0], device_svd=ops_on_gpu)
    else:
        ops = K.Operators(prob.p, device_svd=ops_on_gpu)
    t_ops = time.perf_counter() - t0
    tree = trees[0]
    info = tree.info()
    dev = torch.device("cuda:0")
    qs = [torch.as_tensor(p.charges, dtype=torch.float64, device=dev) for p in probs]
    n_total = sum(p.n for p in probs)
    n_rhs = prob.charges.shape[0]
    n = prob.n

    def evaluate_all(precision, outs):
        if batch:
            K.evaluate_batch(trees, ops, [q[0] for q in qs], precision=precision, outs=outs)
        else:
            K.evaluate(tree, ops, qs[0], precision=precision, out=outs[0])

    def run_graph(precision, steps, warmup):
        """Timed replays of the captured evaluation on a non-default stream."""
        stream = torch.cuda.Stream()
        if batch:
            outs = [torch.empty(p.n, dtype=torch.float64, device=dev) for p in probs]
        else:
            outs = [torch.empty((n_rhs, n), dtype=torch.float64, device=dev)]
        with torch.cuda.stream(stream):
            for _ in range(max(1, warmup)):
                evaluate_all(precision, outs)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            for _ in range(steps):
                evaluate_all(precision, outs)
            torch.cuda.synchronize()
            tb = time.perf_counter()
        return (tb - ta) / steps

    def run(precision, steps, warmup):
        if batch:
            outs = [torch.empty(p.n, dtype=torch.float64, device=dev) for p in probs]
        else:
            outs = [torch.empty((n_rhs, n), dtype=torch.float64, device=dev)]
        for _ in range(warmup):
            evaluate_all(precision, outs)
        torch.cuda.synchronize()
        K.phase_times()
        K.set_profiling(True)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for _ in range(steps):
            evaluate_all(precision, outs)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        K.set_profiling(False)
        ph = K.phase_times()
        return [o.reshape(-1, o.shape[-1]).cpu().numpy() for o in outs], (tb - ta) / steps, ph

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    precision = args.precision or DEFAULT_PRECISION[args.config]
    tuning = None
    if not args.no_autotune:
        # the layout search times graph replays of this very evaluation; an
        # explicit --m2l-tile / --near-fork / --m2l-pair-fill is its start
        from paper_2303_08394_amd import autotune as A
        ts = torch.cuda.Stream()
        touts = ([torch.empty(p.n, dtype=torch.float64, device=dev) for p in probs] if batch
                 else [torch.empty((n_rhs, n), dtype=torch.float64, device=dev)])

        def tune_run():
            with torch.cuda.stream(ts):
                evaluate_all(precision, touts)

        t0 = time.perf_counter()
        tr = A.search(tune_run, ts)
        tuning = {"chosen": tr.best, "start_ms": tr.start_ms, "best_ms": tr.best_ms,
                  "trials": len(tr.trials), "search_s": time.perf_counter() - t0}
        del touts
    layout = {k: K.get_tuning(k) for k in ("m2l_tile_cols", "m2l_split", "m2l_pair_fill", "near_fork", "m2l_async")}
    res, t_eager, phases = run(precision, args.steps, args.warmup)
    result = {"eager_profiled_ms_per_step": t_eager * 1e3, "layout": layout}
    if tuning is not None:
        result["tuning"] = tuning
    t_step = run_graph(precision, args.steps, args.warmup) if not args.no_graph else t_eager
    if not args.no_fp64_leg and precision != "fp64" and args.config != "multi_rhs_1m":
        if tuning is not None:
            # the FP64 path at its own fastest layout (its M2L runs other
            # kernels), then the mixed mode's layout again
            touts = ([torch.empty(p.n, dtype=torch.float64, device=dev) for p in probs] if batch
                     else [torch.empty((n_rhs, n), dtype=torch.float64, device=dev)])

            def tune_run64():
                with torch.cuda.stream(ts):
                    evaluate_all("fp64", touts)

            result["fp64_layout"] = A.search(tune_run64, ts).best
            del touts
        ref, t64, ph64 = run("fp64", max(2, args.steps // 4), 1)
        if not args.no_graph:
            t64 = run_graph("fp64", max(2, args.steps // 4), 1)
        if tuning is not None:
            for k, v in tuning["chosen"].items():
                K.set_tuning(k, v)
        result["fp64_ms_per_step"] = t64 * 1e3
        result["speedup_vs_fp64"] = t64 / t_step
        result["rel_l2_vs_fp64_gpu"] = rel(np.concatenate([r.ravel() for r in res]),
                                           np.concatenate([r.ravel() for r in ref]))
    elif not args.no_fp64_leg and precision != "fp64":
        # multi-RHS: the FP64 reference runs once (it takes seconds at p = 10)
        ref, t64, ph64 = run("fp64", 1, 0)
        result["fp64_ms_per_step"] = t64 * 1e3
        result["speedup_vs_fp64"] = t64 / t_step
        result["rel_l2_vs_fp64_gpu"] = rel(res[0], ref[0])
    # direct sum on a seeded sample of targets (first problem, first charge vector)
    idx = I.sample_indices(n, args.direct_sample)
    ta = time.perf_counter()
    exact = direct.direct(prob.points, prob.charges[0], prob.points[idx], kappa=kappa)
    t_direct = time.perf_counter() - ta
    result["rel_l2_vs_direct_sample"] = rel(res[0][0][idx], exact)
    result["direct_sample"] = {"targets": int(len(idx)), "cpu_s": t_direct}
    if args.config == "plain_20k":
        from oracle import kifmm as OK
        from oracle.octree import Octree
        want = OK.KIFMM(Octree(prob.points, prob.points, uniform_depth=prob.uniform_depth,
                               center=prob.center, halfwidth=prob.halfwidth), prob.p).evaluate(prob.charges)
        result["rel_l2_vs_oracle"] = rel(res[0], want)
        result["oracle_rel_l2_vs_direct"] = rel(want[0], direct.direct(prob.points, prob.charges[0], prob.points))

    # roofline of the dominant kernel
    nrun = args.steps
    ms = {k: v[0] / nrun for k, v in phases.items()}
    launches = {k: v[1] / nrun for k, v in phases.items()}
    dom = max(ms, key=ms.get)
    pn = ops.n
    v_pairs = near_pairs = far_pairs = 0
    for t in trees:
        w = _work_counts(t, pn)
        v_pairs += w[0]
        near_pairs += w[1]
        far_pairs += w[2]
    flops_m2l = 2.0 * pn * pn * v_pairs * n_rhs
    leaf_pairs = (near_pairs + far_pairs) * n_rhs
    pair_stage = launches.get("m2l_pair", 0.0) > 0
    # the split M2L runs the LDS-staged kernel for tiles of up to 160 columns
    # with FP32 sums (below m2l_fp64_sum_min_p); with FP64 sums, up to 96
    # columns in 128-row blocks or 64 in 160-row blocks; otherwise gemm_kernel
    ld = (pn + 31) // 32 * 32
    rows = K.get_tuning("m2l_rows") or (128 if (ld + 127) // 128 * 128 < (ld + 159) // 160 * 160 else 160)
    fp64_sums = prob.p >= K.get_tuning("m2l_fp64_sum_min_p")
    async_m2l = (layout["m2l_async"] == 1
                 and layout["m2l_tile_cols"] <= ((96 if rows == 128 else 64) if fp64_sums else 160))
    if dom == "m2l_pair" or (dom == "m2l" and pair_stage):
        # sparse (adaptive) problems run M2L pair by pair: the algorithmic
        # flops over the whole M2L stage (gathered tiles, pair tiles, pair sums)
        m2l_kind = precision.split("m2l_")[-1]
        peak = {"fp64": PEAK_FP64_MFMA, "fp32": PEAK_FP32_MFMA,
                "bf16x3": PEAK_BF16_MFMA, "bf16x5": PEAK_BF16_MFMA, "f16x3": PEAK_BF16_MFMA}[m2l_kind]
        issued = {"fp64": 1, "fp32": 1, "bf16x3": 3, "bf16x5": 5, "f16x3": 3}[m2l_kind]
        t_stage = (ms["m2l"] + ms["m2l_pair"]) * 1e-3
        gk = "m2l_async_kernel" if m2l_kind in ("bf16x3", "f16x3") and async_m2l else "gemm_kernel"
        roof = {"kernel": f"M2L stage ({gk} gathered + pair tiles, m2l_pair_sum_kernel)",
                "bound": "mfma", "achieved": flops_m2l / t_stage / 1e12, "peak": peak / 1e12,
                "unit": "TFLOP/s", "issued_frac": issued * flops_m2l / t_stage / peak}
    elif dom == "m2l":
        # algorithmic flops (one product per V-list pair), against the peak of
        # the instruction the path issues; split-BF16 issues 3 (5) products
        m2l_kind = precision.split("m2l_")[-1]
        peak = {"fp64": PEAK_FP64_MFMA, "fp32": PEAK_FP32_MFMA,
                "bf16x3": PEAK_BF16_MFMA, "bf16x5": PEAK_BF16_MFMA, "f16x3": PEAK_BF16_MFMA}[m2l_kind]
        issued = {"fp64": 1, "fp32": 1, "bf16x3": 3, "bf16x5": 5, "f16x3": 3}[m2l_kind]
        name = "m2l_async_kernel" if m2l_kind in ("bf16x3", "f16x3") and async_m2l else "gemm_kernel"
        roof = {"kernel": f"{name} (M2L)", "bound": "mfma",
                "achieved": flops_m2l / (ms["m2l"] / launches["m2l"] * 1e-3) / 1e12,
                "peak": peak / 1e12, "unit": "TFLOP/s",
                "issued_frac": issued * flops_m2l / (ms["m2l"] / launches["m2l"] * 1e-3) / peak}
    elif dom == "near":
        roof = {"kernel": "p2p_kernel (near field)", "bound": "alu",
                "achieved": near_pairs * n_rhs / (ms["near"] / launches["near"] * 1e-3) / 1e12,
                "peak": PEAK_PAIRS / 1e12, "unit": "Tpairs/s"}
    elif dom == "far" and ms.get("near", 0.0) == 0.0:
        roof = {"kernel": "p2p_kernel (near + far field)", "bound": "alu",
                "achieved": leaf_pairs / (ms["far"] / launches["far"] * 1e-3) / 1e12,
                "peak": PEAK_PAIRS / 1e12, "unit": "Tpairs/s"}
    else:
        roof = {"kernel": dom, "bound": "alu", "achieved": None, "peak": None, "unit": None}
    roof["frac"] = roof["achieved"] / roof["peak"] if roof["peak"] else None
    # the particle kernels, reported beside the dominant one
    if ms.get("near", 0.0) > 0.0:
        near_rate = near_pairs * n_rhs / (ms["near"] / max(launches["near"], 1) * 1e-3)
        result["near_field"] = {"pairs_per_s": near_rate, "frac_of_valu_peak": near_rate / PEAK_PAIRS,
                                "frac_of_min_op_bound": near_rate / PEAK_PAIRS_MIN_OPS}
    else:
        # near and far field of the leaves in one kernel (the "far" phase)
        leaf_rate = leaf_pairs / (ms["far"] / max(launches["far"], 1) * 1e-3)
        result["leaf_field"] = {"kernel": "p2p_kernel (near + far field)", "pairs_per_s": leaf_rate,
                                "frac_of_valu_peak": leaf_rate / PEAK_PAIRS,
                                "frac_of_min_op_bound": leaf_rate / PEAK_PAIRS_MIN_OPS}
    # the equivalent-density solves (FP64 GEMMs in every mode) and the
    # translations (FP32 GEMMs in the FP32-bulk modes, FP64 in the FP64
    # ones): algorithmic flops (2 n^2 per box column) over the phase's time
    # per evaluation, all levels' launches together
    cols = np.zeros(4, np.int64)
    for t in trees:
        cols += np.array(_translation_counts(t), np.int64)
    fp64_bulk = precision.startswith("fp64")
    trans = {}
    for k, name, c, pk in (("uc2e", "gemm_kernel<FP64>", cols[0], PEAK_FP64_MFMA),
                           ("dc2e", "gemm_kernel<FP64>", cols[1], PEAK_FP64_MFMA),
                           ("m2m", "gemm_kernel<FP64>" if fp64_bulk else "gemm_kernel<FP32> + m2m_sum_kernel",
                            cols[2], PEAK_FP64_MFMA if fp64_bulk else PEAK_FP32_MFMA),
                           ("l2l", "gemm_kernel<FP64>" if fp64_bulk else "gemm_kernel<FP32>",
                            cols[3], PEAK_FP64_MFMA if fp64_bulk else PEAK_FP32_MFMA)):
        if ms.get(k, 0.0) > 0.0:
            flops = 2.0 * pn * pn * float(c) * n_rhs
            ach = flops / (ms[k] * 1e-3)
            trans[k] = {"kernel": name, "launches": launches[k], "flop": flops, "ms": ms[k],
                        "achieved_tflops": ach / 1e12, "peak_tflops": pk / 1e12, "frac": ach / pk}
    result["translation_rooflines"] = trans
    # the committed counter summaries are per M2L tile width (two parity parts
    # per tile, gathered tiles: the layouts whose M2L kernel they measured)
    m2l_counters = (args.config == "uniform_1m" and dom == "m2l" and layout["m2l_split"] == 1
                    and layout["m2l_pair_fill"] != 101)
    sfx = (precision + ("" if layout["m2l_tile_cols"] == 64 else f"_tile{layout['m2l_tile_cols']}")
           + ("" if layout["m2l_async"] else "_regstaged"))
    roof["traffic"] = _measured_traffic(sfx) if m2l_counters else None
    if m2l_counters:
        # SQ_VALU_MFMA_BUSY_CYCLES over the launch's cycles, and the clock the
        # GRBM counter reads meanwhile (rocprofv3, same kernel source)
        roof["mfma_busy_counter"] = _profile_value("m2l_mfma_util_uniform1m_p6.txt", f"m2l_mfma_busy_{sfx}")
        roof["clock_ghz_counter"] = _profile_value("m2l_mfma_util_uniform1m_p6.txt", f"m2l_clock_ghz_{sfx}")

    if not batch and n_rhs == 1 and not args.no_gradient and not kappa:
        # potentials + gradients (kifmm_evaluate_gradient), graph replays as
        # above, against the FP64 gradient on the same tree
        def grad_run(prec, steps):
            out = torch.empty((1, 4, n), dtype=torch.float64, device=dev)
            stream = torch.cuda.Stream()
            with torch.cuda.stream(stream):
                for _ in range(2):
                    K.evaluate_gradient(tree, ops, qs[0], precision=prec, out=out)
                torch.cuda.synchronize()
                ta = time.perf_counter()
                for _ in range(steps):
                    K.evaluate_gradient(tree, ops, qs[0], precision=prec, out=out)
                torch.cuda.synchronize()
                tb = time.perf_counter()
            return out.cpu().numpy()[0], (tb - ta) / steps
        g, tg = grad_run(precision, args.steps)
        g64, _ = grad_run("fp64", 1)
        result["gradient"] = {"ms_per_step": tg * 1e3, "Mpoints_per_s": n / tg / 1e6,
                              "rel_l2_vs_fp64_gpu": rel(g[1:], g64[1:])}

    if not batch:
        # the tree's points re-sorted on the device after each point moves to
        # a fresh position inside its leaf (kifmm_tree_update_points), against
        # the host build above; the original points are put back afterwards
        bx, inf = tree.boxes(), tree.info()
        sperm, _ = tree.perm()
        lo = np.asarray(inf.root_center) - inf.root_halfwidth
        u = np.random.default_rng(7).random((inf.n_src, 3))
        moved = np.empty((inf.n_src, 3))
        for b in np.nonzero(bx["is_leaf"] == 1)[0]:
            s0, s1 = bx["src_range"][b]
            if s1 > s0:
                idx = sperm[s0:s1]
                w = 2 * inf.root_halfwidth / 2 ** int(bx["level"][b])
                moved[idx] = lo + (bx["anchor"][b] + u[idx]) * w
        x_new = torch.as_tensor(moved, dtype=torch.float64, device=dev)
        x_old = torch.as_tensor(prob.points, dtype=torch.float64, device=dev)
        tree.update_points(x_new)
        tree.update_points(x_old)
        ta = time.perf_counter()
        for _ in range(3):
            tree.update_points(x_new)
            tree.update_points(x_old)
        result["tree_update_ms"] = (time.perf_counter() - ta) / 6 * 1e3

    line = {
        "metric": "FMM evaluate Mpoints/s at 1M pts p=6, rel L2 err<=1e-5; mixed vs plain FP64",
        "value": n_total / t_step / 1e6,
        "unit": "Mpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16x3": "f32+bf16x3", "bf16x5": "f32+bf16x5", "f16x3": "f32+f16x3",
                  "fp64": "f64", "fp64+m2l_fp32": "f64+f32", "fp64+m2l_f16x3": "f64+f16x3"}[precision],
        "data": "synthetic",
        "config": {"workload": (prob.name + (f"_screened_kappa{kappa:g}" if kappa else "")) if not batch
                   else f"batch of {len(probs)} problems",
                   "n_points": n_total, "n_rhs": n_rhs, "p": prob.p,
                   "depth": max(t.info().depth for t in trees),
                   "leaves": sum(t.info().n_leaves for t in trees), "precision": precision},
        "roofline": roof,
        "phases_ms": {k: round(v, 4) for k, v in ms.items()},
        "launches_per_step": {k: v for k, v in launches.items()},
        "work": {"m2l_flop": flops_m2l, "v_pairs": v_pairs, "near_pairs": near_pairs,
                 "leaf_far_pairs": far_pairs},
        "tree_build_s": t_tree,
        "precompute_svd": "gpu" if ops_on_gpu else "host",
        "precompute_s": t_ops,
        **result,
    }
    if args.config == "paper_sphere_1m":
        # the paper quotes mean list sizes |U|=11, |V|=42, |X|=3, |W|=3 for its tree
        bx = tree.boxes()
        leaves = int((bx["is_leaf"] == 1).sum())
        lvl2 = int((bx["level"] >= 2).sum())
        line["list_means"] = {"U": info.n_u / leaves, "V": info.n_v / lvl2, "W": info.n_w / leaves,
                              "X": info.n_x / lvl2}
    if not args.no_cpu_baseline:
        if args.config == "uniform_1m":
            line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
