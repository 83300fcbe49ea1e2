"""Autotuner for the predictor's knobs, by measured throughput on the GPU.

Knobs: epoch size (the unit of batch-synchronous work, a "chunk"), the length
of a call's first epoch (a short one fills the table early), table size
(log2 entries), ways, origin / direction quantisation bits, the number of
failing lanes at which a prediction wave traverses at once instead of
queueing (a pure scheduling knob: results do not depend on it), and the BVH's
leaf size (given a function that builds the tree for a leaf size; each size is
built once and its plain traversal is the reference for the skip constraint).  The traversal
stack depth is not a knob: the per-lane stack holds the deepest tree the
library accepts (64 levels), which is what makes overflow impossible.  Every configuration the tuner
can pick is an ordinary predictor configuration, traced by the same kernels
that the parity tests check against the oracle.

Search: coordinate descent from a start point, one knob at a time over its
candidate list, for `rounds` passes; each point is timed with HIP events
(median of `reps` runs, each run = predictor reset + trace).  With `warm_rays`
(the rays of an earlier frame of the same view) each run first traces those,
untimed, after the reset, so that the timed trace sees the tables a renderer
would carry from frame to frame.  Optionally a minimum fraction of skipped
nodes can be imposed, so that the tuner does not trade all prediction away
for speed.
"""
from __future__ import annotations

import statistics
from dataclasses import dataclass, field

import torch

from . import hrpp

DEFAULT_SPACE = {
    "epoch_rays": [1 << 15, 1 << 16, 1 << 17, 1 << 18, 1 << 19, 1 << 20, 1 << 21, 1 << 22],
    "log2_entries": [16, 18, 20, 22],
    "ways": [4, 8],
    "origin_bits": [3, 4, 5, 6, 7],
    "dir_bits": [3, 4, 5, 6, 7],
    "inline_lanes": [16, 32, 48, 56, 64, 65],
    "first_epoch_rays": [0, 1 << 16, 1 << 17, 1 << 18, 1 << 19],
    "leaf_max": [1, 2, 3, 4],
}


@dataclass
class TuneResult:
    best: dict
    best_ms: float
    best_stats: dict
    trials: list = field(default_factory=list)


def _time_config(bvh, rays, query, mode, cfg, reps, plain_nodes, warm_rays=None):
    pred = hrpp.Predictor(bvh, **cfg)
    out = (torch.empty(rays.shape[0], dtype=torch.uint8, device=rays.device) if query == "any"
           else torch.empty((rays.shape[0], 4), dtype=torch.float32, device=rays.device))
    wout = None
    if warm_rays is not None:
        wout = (torch.empty(warm_rays.shape[0], dtype=torch.uint8, device=rays.device) if query == "any"
                else torch.empty((warm_rays.shape[0], 4), dtype=torch.float32, device=rays.device))

    def trace(r, o, stats=None):
        if query == "any":
            hrpp.trace_anyhit(bvh, pred, r, out=o, stats=stats)
        else:
            hrpp.trace_closest(bvh, pred, r, mode=mode, out=o, stats=stats)

    def prepare():
        # untimed: the tables of the earlier frame
        if warm_rays is not None:
            pred.reset()
            trace(warm_rays, wout)

    def run(stats=None):
        # timed: reset + trace, or (warm) the trace alone
        if warm_rays is None:
            pred.reset()
        trace(rays, out, stats)

    prepare()
    run()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        prepare()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        run()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    st = hrpp.new_stats()
    prepare()
    run(st)
    torch.cuda.synchronize()
    s = hrpp.stats_dict(st)
    s["pct_nodes_skipped"] = 100.0 * (1.0 - s["nodes_visited"] / plain_nodes) if plain_nodes else 0.0
    del pred
    return statistics.median(times), s


def tune(bvh, rays, query: str = "any", mode: str = "paper", start: dict | None = None,
         space: dict | None = None, rounds: int = 2, reps: int = 3, min_skip_pct: float | None = None,
         knobs=("epoch_rays", "log2_entries", "ways", "origin_bits", "dir_bits"), log=None,
         warm_rays=None) -> TuneResult:
    """Coordinate-descent search of the predictor configuration minimising trace time.

    `bvh` is a BVH, or a function from a leaf size to a BVH over the same
    triangles; the latter is required to tune "leaf_max", and the returned
    configuration then carries the chosen "leaf_max" next to the predictor's
    knobs."""
    space = dict(DEFAULT_SPACE, **(space or {}))
    tree_fn = bvh if callable(bvh) else None
    if "leaf_max" in knobs and tree_fn is None:
        raise ValueError("tuning leaf_max needs a function from a leaf size to a BVH")
    cfg = dict(log2_entries=20, ways=8, origin_bits=5, dir_bits=6, epoch_rays=1 << 19)
    if tree_fn is not None:
        cfg["leaf_max"] = 4
    if start:
        cfg.update(start)
    trees, plain = {}, {}

    def tree_of(c):
        # the tree and its plain node count (for the skip constraint and the report)
        leaf = c.get("leaf_max") if tree_fn is not None else None
        if leaf not in trees:
            t = tree_fn(leaf) if tree_fn is not None else bvh
            st = hrpp.new_stats()
            if query == "any":
                hrpp.trace_anyhit(t, None, rays, stats=st)
            else:
                hrpp.trace_closest(t, None, rays, mode=mode, stats=st)
            torch.cuda.synchronize()
            trees[leaf], plain[leaf] = t, hrpp.stats_dict(st)["nodes_visited"]
        return trees[leaf], plain[leaf]

    seen = {}
    trials = []

    def evaluate(c):
        key = tuple(sorted(c.items()))
        if key not in seen:
            t, plain_nodes = tree_of(c)
            pc = {k: v for k, v in c.items() if k != "leaf_max"}
            ms, s = _time_config(t, rays, query, mode, pc, reps, plain_nodes, warm_rays)
            ok = min_skip_pct is None or s["pct_nodes_skipped"] >= min_skip_pct
            seen[key] = (ms, s, ok)
            trials.append(dict(config=dict(c), ms=ms, pct_nodes_skipped=s["pct_nodes_skipped"], feasible=ok))
            if log:
                log(f"autotune {c} -> {ms:.3f} ms, {s['pct_nodes_skipped']:.1f}% skipped{'' if ok else ' (rejected)'}")
        return seen[key]

    best_ms, best_s, best_ok = evaluate(cfg)
    for _ in range(rounds):
        changed = False
        for knob in knobs:
            for v in space[knob]:
                c = dict(cfg, **{knob: v})
                if c.get("first_epoch_rays", 0) > c["epoch_rays"]:
                    continue                          # not a valid predictor
                ms, s, ok = evaluate(c)
                if ok and (not best_ok or ms < best_ms):
                    cfg, best_ms, best_s, best_ok, changed = c, ms, s, True, True
        if not changed:
            break
    return TuneResult(best=cfg, best_ms=best_ms, best_stats=best_s, trials=trials)
