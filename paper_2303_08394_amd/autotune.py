"""Measured choice of an evaluation's launch layout.

The layout knobs of ``kifmm_set_tuning`` change how an evaluation is cut into
kernel launches, not the method: the M2L tile width (64, 96, 128, 160 or 192 output
columns per block; results bitwise equal), whether each M2L tile runs as one
block or as two parity parts, the tile-fill threshold below which a problem's
M2L runs pair by pair, where the near field sits in the schedule, and the
shape of the M2L block (160 or 128 operator rows; for 128-column split tiles
the kernel with 80 x 64 wave tiles; results bitwise equal) and the staging of
the split M2L kernel (straight into LDS or through registers; bitwise equal).  Which
layout is fastest depends on the workload (uniform or adaptive tree, points
per leaf, order p, right-hand sides) and on the device, so it is measured:
``search`` times each candidate on the caller's own evaluation, with HIP events
on the evaluation stream around graph replays as the library runs them, walks
the knobs one at a time (coordinate descent), keeps a candidate only if it is
faster by a margin, confirms a changed layout against the starting one by
alternate re-timing, and leaves the fastest layout in force.  Results can be
kept in a JSON file keyed by a workload signature, so a later process applies
them without timing.

The knobs are process-wide: a search changes them for every later evaluation
in the process, which is the point.  Concurrent evaluations during a search
are timed with it.
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass, field
from typing import Callable, Optional, Sequence, Tuple

from . import kifmm as K

# The searched knobs and their candidates, in search order.  The first
# candidate of each is its library default.
SPACE: Tuple[Tuple[str, Tuple[int, ...]], ...] = (
    ("m2l_tile_cols", (64, 96, 128, 160, 192)),
    # the split M2L kernel: staging straight into LDS (1) or through registers
    ("m2l_async", (1, 0)),
    ("m2l_split", (1, 0)),
    ("m2l_pair_fill", (40, 0, 101)),
    ("near_fork", (4, 2, 0)),
    # the M2L block's shape: operator rows per block (0: fewest padded rows),
    # and for 128-column split tiles the wide-tile kernel (80 x 64 wave tiles)
    ("m2l_rows", (0, 160, 128)),
    ("m2l_wide", (0, 1)),
)


@dataclass
class TuneResult:
    best: dict  # knob -> value left in force
    best_ms: float  # time per evaluation with it (None when applied from a cache)
    start_ms: Optional[float]  # with the values in force when the search began
    trials: list = field(default_factory=list)  # (setting, ms) in the order timed
    from_cache: bool = False


def _timed(run: Callable[[], None], stream, n: int) -> float:
    import torch

    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(n):
        run()
    t1.record(stream)
    t1.synchronize()
    return t0.elapsed_time(t1) / n


def time_ms(run: Callable[[], None], stream, steps: int = 30, warmup: int = 3, budget_s: float = 0.25) -> float:
    """Mean time of one ``run()`` in ms, between HIP events recorded on
    ``stream`` (the stream ``run`` launches on).  The warm-up calls absorb
    plan rebuilds and graph captures that a knob change triggers; one timed
    call then sizes the sample to about ``budget_s`` seconds (between 2 and
    ``steps`` calls), so slow workloads are not timed for minutes."""
    for _ in range(warmup):
        run()
    stream.synchronize()
    one = _timed(run, stream, 1)
    n = max(2, min(steps, int(budget_s * 1e3 / max(one, 1e-3))))
    return _timed(run, stream, n)


def _apply(setting: dict, set_: Callable[[str, int], None]):
    for k, v in setting.items():
        set_(k, v)


def search(run: Callable[[], None], stream=None, *, space: Sequence = SPACE, steps: int = 30,
           warmup: int = 3, budget_s: float = 0.25, min_gain: float = 0.03, confirm: int = 3,
           timer: Optional[Callable[[], float]] = None,
           get: Callable[[str], int] = K.get_tuning, set_: Callable[[str, int], None] = K.set_tuning
           ) -> TuneResult:
    """Coordinate descent over ``space``: for each knob in turn, time every
    candidate with the other knobs at their current best, and keep the
    fastest if it beats the best so far by more than ``min_gain`` (a
    fraction; it keeps run-to-run noise from moving the layout).  A layout
    that differs from the starting one is then confirmed: both are timed
    ``confirm`` more times, alternately, and the new one is kept only if its
    median still beats the start's by ``min_gain``.  The kept layout is left
    in force; on an error the starting layout is put back.  ``timer``
    (default: ``time_ms(run, stream, steps, warmup, budget_s)``) returns ms per
    evaluation under the knobs in force."""
    if timer is None:
        if stream is None:
            raise ValueError("search: a stream (the one run() launches on) or a timer is required")
        timer = lambda: time_ms(run, stream, steps, warmup, budget_s)  # noqa: E731
    cur = {k: get(k) for k, _ in space}
    first = dict(cur)
    try:
        start = timer()
        best_ms = start
        trials = [(dict(cur), start)]
        for k, cands in space:
            keep = cur[k]
            for v in cands:
                if v == cur[k]:
                    continue
                set_(k, v)
                t = timer()
                trials.append(({**cur, k: v}, t))
                if t < best_ms * (1.0 - min_gain):
                    best_ms, keep = t, v
            set_(k, keep)
            cur[k] = keep
        if cur != first and confirm > 0:
            ts_first, ts_best = [], []
            for _ in range(confirm):
                _apply(first, set_)
                ts_first.append(timer())
                trials.append((dict(first), ts_first[-1]))
                _apply(cur, set_)
                ts_best.append(timer())
                trials.append((dict(cur), ts_best[-1]))
            med_first = sorted(ts_first)[len(ts_first) // 2]
            med_best = sorted(ts_best)[len(ts_best) // 2]
            if med_best < med_first * (1.0 - min_gain):
                best_ms = med_best
            else:
                cur, best_ms = dict(first), med_first
                _apply(cur, set_)
    except BaseException:
        _apply(first, set_)
        raise
    return TuneResult(best=dict(cur), best_ms=best_ms, start_ms=start, trials=trials)


def signature(tree: "K.Tree", ops: "K.Operators", precision: str, n_rhs: int = 1, what: str = "evaluate") -> str:
    """Workload key for the cache: tree shape, order, precision, right-hand
    sides, the kind of call, and the device."""
    import torch

    i = tree.info()
    dev = torch.cuda.get_device_name(torch.cuda.current_device()) if torch.cuda.is_available() else "none"
    parts = [what, f"src{i.n_src}", f"tgt{i.n_tgt}", f"boxes{i.n_boxes}", f"leaves{i.n_leaves}",
             f"depth{i.depth}", f"v{i.n_v}", f"p{ops.p}", precision, f"rhs{n_rhs}", dev]
    return "|".join(str(x) for x in parts)


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def autotune(run: Callable[[], None], stream, *, key: Optional[str] = None,
             cache_path: Optional[str] = None, **kw) -> TuneResult:
    """``search`` with an optional JSON cache: a cached layout for ``key`` is
    applied without timing; a new result is stored under ``key``."""
    if cache_path and key:
        hit = _load(cache_path).get(key)
        if isinstance(hit, dict) and hit:
            set_ = kw.get("set_", K.set_tuning)
            for k, v in hit.items():
                set_(k, int(v))
            return TuneResult(best={k: int(v) for k, v in hit.items()}, best_ms=None, start_ms=None,
                              from_cache=True)
    res = search(run, stream, **kw)
    if cache_path and key:
        d = _load(cache_path)
        d[key] = res.best
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return res


def autotune_evaluate(tree: "K.Tree", ops: "K.Operators", charges, precision: str = "fp32", *,
                      stream=None, cache_path: Optional[str] = None, **kw) -> TuneResult:
    """Tune the layout for ``evaluate(tree, ops, charges, precision)`` on
    ``stream`` (a new stream when None: the library replays graphs only on
    non-default streams)."""
    import torch

    if stream is None:
        stream = torch.cuda.Stream()
    q = charges
    n_rhs = 1 if q.dim() == 1 else int(q.shape[0])
    shape = (tree.info().n_tgt,) if q.dim() == 1 else (n_rhs, tree.info().n_tgt)
    out = torch.empty(shape, dtype=q.dtype, device=q.device)

    def run():
        K.evaluate(tree, ops, q, precision, out=out, stream=stream)

    return autotune(run, stream, key=signature(tree, ops, precision, n_rhs), cache_path=cache_path, **kw)
