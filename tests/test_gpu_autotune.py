"""The autotuner returns the fastest feasible configuration it timed."""
from __future__ import annotations

import pytest

import scenegen as sg

pytestmark = pytest.mark.gpu


def test_autotune_small_space():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_01304_amd as hrpp
    from paper_1910_01304_amd import autotune
    print("[gpu-case] autotune tiny", flush=True)
    tris, rays = sg.tiny_workload()
    bvh = hrpp.BVH(tris)
    r = torch.from_numpy(rays).cuda()
    space = {"epoch_rays": [64, 256, 1024], "log2_entries": [10, 12], "ways": [4], "origin_bits": [4, 5],
             "dir_bits": [5, 6]}
    res = autotune.tune(bvh, r, query="any", start=dict(log2_entries=12, ways=4, origin_bits=5, dir_bits=6,
                                                          epoch_rays=256), space=space, rounds=2, reps=2)
    for k, v in res.best.items():
        assert v in space[k], (k, v)
    feasible = [t["ms"] for t in res.trials if t["feasible"]]
    assert res.best_ms == min(feasible)
    # a skip constraint nobody can meet leaves every trial infeasible but still returns a config
    res2 = autotune.tune(bvh, r, query="any", start=res.best, space=space, rounds=1, reps=1, min_skip_pct=101.0,
                         knobs=("epoch_rays",))
    assert all(not t["feasible"] for t in res2.trials)
