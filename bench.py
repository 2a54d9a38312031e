#!/usr/bin/env python3
"""Benchmark of the KIFMM evaluation on one MI355X.

A step is one full evaluation (gather, P2M, M2M, UC2E, P2L, M2L, L2L, DC2E,
the fused L2P + M2P + near-field leaf kernel, scatter) of the 1M-point
uniform-cube workload (p = 6, uniform depth 5, charges in [-1, 1)) with the
tree, the operators and the charges already resident in HBM.  The headline
is the mixed-precision path (FP32 bulk arithmetic, FP64 check-to-equivalent
solves and FP64 per-target sums); the plain FP64 path runs on the same tree
as the comparison leg, and its result is the reference of the reported error.

Prints one JSON line.  --gpus N with N > 1 exits: this build runs on one GPU.
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
PEAK_BF16_MFMA = 2.5e15     # dense BF16 matrix FLOP/s
PEAK_HBM = 8.0e12
# The particle kernels are bound by plain FP32 VALU issue: 256 CUs x 4 SIMDs x
# 16 lanes x 2.4 GHz = 3.93e13 lane-instructions/s.  One pair interaction issues
# 9 full-rate instructions (3 sub, mul + 2 fma for r^2, select, fma for the sum)
# plus one reciprocal square root at quarter rate (4 issue slots): 13 slots.
VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9
SLOTS_PER_PAIR = 13.0
PEAK_PAIRS = VALU_LANE_OPS / SLOTS_PER_PAIR


def _workload(args):
    from paper_2303_08394_amd import inputs as I
    if args.config == "uniform_1m":
        return I.uniform_1m()
    if args.config == "uniform_20k":
        return I.plain_fp64_20k()
    raise SystemExit(f"unknown config {args.config}")


def cpu_baseline():
    """The FP64 oracle, single-threaded, on a bounded sample of the same
    recipe: N = 125,000 uniform-cube points with uniform depth 4 (the same
    ~30.5 points per leaf and p = 6 as the 1M workload)."""
    from threadpoolctl import threadpool_limits

    from oracle import kifmm as OK
    from oracle.octree import Octree
    from paper_2303_08394_amd import inputs as I
    n = 125_000
    x, q = I.uniform_cube(n, seed=0, charge_range=(-1.0, 1.0))
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        tree = Octree(x, x, uniform_depth=4, center=I.UNIT_CUBE_CENTER, halfwidth=I.UNIT_CUBE_HALFWIDTH)
        fm = OK.KIFMM(tree, 6)
        t1 = time.perf_counter()
        fm.evaluate(q[0])
        t2 = time.perf_counter()
    ev = t2 - t1
    return {"value": n / ev / 1e6, "unit": "Mpoints/s", "cores": 1, "kind": "oracle",
            "sample": f"FP64 oracle evaluate, N={n} uniform cube, depth 4 (30.5 pts/leaf), "
                      f"p=6, one BLAS thread; evaluate {ev:.1f} s, tree+lists {t1 - t0:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="uniform_1m")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16x3", "bf16x5", "fp64"])
    ap.add_argument("--no-fp64-leg", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--direct-sample", type=int, default=200)
    ap.add_argument("--m2l-tile", type=int, default=0, help="M2L output columns per block (64/128)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build evaluates on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU partition is described in DESIGN.md, not built)", file=sys.stderr)
        return 2

    import torch

    from oracle import direct
    from paper_2303_08394_amd import inputs as I
    from paper_2303_08394_amd import kifmm as K

    if args.m2l_tile:
        K.set_tuning("m2l_tile_cols", args.m2l_tile)
    prob = _workload(args)
    t0 = time.perf_counter()
    tree = K.Tree(prob.points, uniform_depth=prob.uniform_depth, ncrit=prob.ncrit,
                  max_depth=prob.max_depth, center=prob.center, halfwidth=prob.halfwidth)
    t_tree = time.perf_counter() - t0
    t0 = time.perf_counter()
    ops = K.Operators(prob.p)
    t_ops = time.perf_counter() - t0
    info = tree.info()
    dev = torch.device("cuda:0")
    q = torch.as_tensor(prob.charges, dtype=torch.float64, device=dev)
    n = prob.n
    stream = torch.cuda.current_stream()

    def run(precision, steps, warmup):
        out = torch.empty((q.shape[0], n), dtype=torch.float64, device=dev)
        for _ in range(warmup):
            K.evaluate(tree, ops, q, precision=precision, out=out)
        torch.cuda.synchronize()
        K.phase_times()
        K.set_profiling(True)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for _ in range(steps):
            K.evaluate(tree, ops, q, precision=precision, out=out)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        K.set_profiling(False)
        ph = K.phase_times()
        return out, (tb - ta) / steps, ph

    out, t_step, phases = run(args.precision, args.steps, args.warmup)
    res = out[0].double().cpu().numpy()
    result = {}
    if not args.no_fp64_leg and args.precision != "fp64":
        ref, t64, ph64 = run("fp64", max(3, args.steps // 4), 1)
        ref = ref[0].cpu().numpy()
        result["fp64_ms_per_step"] = t64 * 1e3
        result["speedup_vs_fp64"] = t64 / t_step
        result["rel_l2_vs_fp64_gpu"] = float(np.linalg.norm(res - ref) / np.linalg.norm(ref))
    idx = I.sample_indices(n, args.direct_sample)
    exact = direct.direct(prob.points, prob.charges[0], prob.points[idx])
    result["rel_l2_vs_direct_sample"] = float(np.linalg.norm(res[idx] - exact) / np.linalg.norm(exact))

    # roofline of the dominant kernel
    nrun = args.steps
    ms = {k: v[0] / nrun for k, v in phases.items()}
    launches = {k: v[1] / nrun for k, v in phases.items()}
    dom = max(ms, key=ms.get)
    pn = ops.n
    v_pairs = info.n_v
    flops_m2l = 2.0 * pn * pn * v_pairs
    # P2P pair interactions of the fused leaf kernel: near field + L2P (+ M2P)
    bx = tree.boxes()
    uoff, uitems = tree.list(K.LIST_U)
    nt = bx["tgt_range"][:, 1] - bx["tgt_range"][:, 0]
    ns = bx["src_range"][:, 1] - bx["src_range"][:, 0]
    leaves = np.nonzero(bx["is_leaf"] == 1)[0]
    near_pairs = 0
    for b in leaves:
        near_pairs += int(nt[b]) * int(ns[uitems[uoff[b]:uoff[b + 1]]].sum())
    woff, witems = tree.list(K.LIST_W)
    far_pairs = int(nt[leaves][bx["level"][leaves] >= 2].sum()) * pn + \
        int(sum(nt[b] * (woff[b + 1] - woff[b]) for b in leaves)) * pn
    leaf_pairs = near_pairs + far_pairs
    if dom == "m2l":
        # algorithmic flops (one product per V-list pair), against the peak of
        # the instruction the path issues; split-BF16 issues 3 (5) products
        peak = {"fp64": PEAK_FP64_MFMA, "fp32": PEAK_FP32_MFMA,
                "bf16x3": PEAK_BF16_MFMA, "bf16x5": PEAK_BF16_MFMA}[args.precision]
        issued = {"fp64": 1, "fp32": 1, "bf16x3": 3, "bf16x5": 5}[args.precision]
        roof = {"kernel": "gemm_kernel (M2L)", "bound": "mfma",
                "achieved": flops_m2l / (ms["m2l"] * 1e-3) / 1e12,
                "peak": peak / 1e12, "unit": "TFLOP/s",
                "issued_frac": issued * flops_m2l / (ms["m2l"] * 1e-3) / peak}
    else:
        roof = {"kernel": f"{dom}", "bound": "alu",
                "achieved": leaf_pairs / (ms["leaf"] * 1e-3) / 1e12,
                "peak": PEAK_PAIRS / 1e12, "unit": "Tpairs/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = None

    line = {
        "metric": "FMM evaluate Mpoints/s at 1M pts p=6, rel L2 err<=1e-5; mixed vs plain FP64",
        "value": n / t_step / 1e6,
        "unit": "Mpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16x3": "bf16x3", "bf16x5": "bf16x5", "fp64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": prob.name, "n_points": n, "p": prob.p, "depth": info.depth,
                   "leaves": info.n_leaves, "precision": args.precision},
        "roofline": roof,
        "phases_ms": {k: round(v, 4) for k, v in ms.items()},
        "launches_per_step": {k: v for k, v in launches.items()},
        "work": {"m2l_flop": flops_m2l, "v_pairs": v_pairs, "u_pairs": info.n_u,
                 "near_pairs": near_pairs, "leaf_far_pairs": far_pairs},
        "tree_build_s": t_tree,
        "precompute_s": t_ops,
        **result,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
