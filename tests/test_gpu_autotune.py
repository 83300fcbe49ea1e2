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


def test_autotune_warm_tables():
    # with warm_rays each timed trace starts from the tables those rays left
    # (the untimed first frame), so even its first epoch finds entries
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_01304_amd as hrpp
    from paper_1910_01304_amd import autotune
    print("[gpu-case] autotune tiny, warm tables", flush=True)
    tris, rays = sg.tiny_workload()
    bvh = hrpp.BVH(tris)
    first, second = torch.from_numpy(rays[:2048]).cuda(), torch.from_numpy(rays[2048:]).cuda()
    space = {"epoch_rays": [256, 4096], "origin_bits": [4, 5], "dir_bits": [5, 6]}
    start = dict(log2_entries=12, ways=4, origin_bits=5, dir_bits=6, epoch_rays=4096)
    res = autotune.tune(bvh, second, query="any", start=start, space=space, rounds=1, reps=2, warm_rays=first)
    for k, v in res.best.items():
        assert k not in space or v in space[k], (k, v)
    assert res.best_ms == min(t["ms"] for t in res.trials if t["feasible"])
    assert res.best_stats["positives"] > 0
    # one epoch over the second half: a reset table predicts nothing, a warm one does
    one_epoch = dict(res.best, epoch_rays=4096)
    st = autotune._time_config(bvh, second, "any", "paper", one_epoch, 1, 1, warm_rays=first)[1]
    st0 = autotune._time_config(bvh, second, "any", "paper", one_epoch, 1, 1)[1]
    assert st["positives"] > 0 and st0["positives"] == 0


def test_autotune_leaf_size():
    # with a tree builder the tuner also picks the leaf size; each size is built
    # once and compared with its own plain traversal
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_01304_amd as hrpp
    from paper_1910_01304_amd import autotune
    print("[gpu-case] autotune tiny, leaf size", flush=True)
    tris, rays = sg.tiny_workload()
    r = torch.from_numpy(rays).cuda()
    built = []

    def tree(leaf):
        built.append(leaf)
        return hrpp.BVH(tris, leaf_max=leaf)

    space = {"leaf_max": [1, 2, 4], "epoch_rays": [256, 1024]}
    start = dict(log2_entries=12, ways=4, origin_bits=5, dir_bits=6, epoch_rays=256, leaf_max=4)
    res = autotune.tune(tree, r, query="any", start=start, space=space, rounds=2, reps=2,
                        knobs=("leaf_max", "epoch_rays"))
    assert res.best["leaf_max"] in space["leaf_max"] and res.best["epoch_rays"] in space["epoch_rays"]
    assert sorted(built) == [1, 2, 4]                      # one tree per leaf size
    assert {t["config"]["leaf_max"] for t in res.trials} == {1, 2, 4}
    assert res.best_ms == min(t["ms"] for t in res.trials if t["feasible"])
    with pytest.raises(ValueError):
        autotune.tune(hrpp.BVH(tris), r, knobs=("leaf_max",))
