"""Batched execution: every job of a batch computes exactly what its own
trace call computes (results, counters, table), with direct launches and
with a captured hipGraph replayed several times."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
import scenegen as sg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hrpp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_01304_amd as h
    h.load_library()
    return h


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _jobs_spec():
    # (scene seed, triangles, rays, query, mode, predictor (T, W, qo, qd, E) or None)
    return [
        (11, 3000, 20000, "any", "paper", (12, 4, 5, 6, 4096)),
        (12, 20000, 9000, "any", "paper", (14, 8, 4, 5, 1000)),
        (13, 700, 30000, "closest", "paper", (13, 8, 5, 6, 2048)),
        (14, 15000, 12345, "closest", "exact", (12, 4, 5, 6, 3000)),
        (15, 5000, 7000, "any", "paper", None),
        (16, 9000, 5000, "closest", "paper", None),
        (17, 1, 100, "any", "paper", (4, 2, 3, 3, 16)),
        (18, 4000, 1, "closest", "paper", (8, 4, 5, 6, 64)),
        # go-up levels >= 1 (predicted subtrees) run as groups of their own
        (19, 6000, 15000, "any", "paper", (12, 4, 5, 6, 2048, 0, 1)),
        (20, 8000, 11000, "closest", "paper", (13, 8, 5, 6, 4096, 0, 2)),
        (21, 3000, 6000, "closest", "exact", (12, 4, 4, 4, 1500, 1, 3)),
        # replacement policies
        (22, 5000, 12000, "any", "paper", (6, 2, 5, 6, 3000, 0, 0, 1, 3)),
        (23, 7000, 9000, "closest", "paper", (7, 4, 5, 6, 2500, 0, 2, 65, 1)),
        # a short first epoch (its rounds differ from the other jobs')
        (24, 6000, 14000, "any", "paper", (12, 8, 5, 6, 8192, 0, 0, 1, 0, 700)),
        (25, 4000, 10000, "closest", "exact", (12, 4, 5, 6, 6000, 0, 0, 0, 0, 1)),
        # epochs of at most 256 rays: one workgroup per job runs all its epochs
        (26, 5000, 3000, "any", "paper", (12, 4, 5, 6, 256)),
        (27, 3000, 2000, "closest", "exact", (12, 4, 5, 6, 100, 0, 1)),
        (28, 4000, 2500, "closest", "paper", (12, 8, 5, 6, 200, 0, 0, 65, 0, 50)),
        (29, 2000, 300, "any", "paper", (10, 4, 5, 6, 1)),
    ]


def _build(hrpp, torch):
    jobs = []
    for seed, ntri, nray, query, mode, pc in _jobs_spec():
        tris = sg.mixed_scene(seed, ntri)
        sh, ao = sg.secondary_rays_on_surface(tris, nray, seed + 100)
        rays = np.concatenate([sh, ao]) if query == "any" else np.concatenate([sh, ao])
        if query == "closest":
            rays[:, 7] = np.inf
        bvh = hrpp.BVH(tris)
        jobs.append(dict(tris=tris, rays_np=rays, bvh=bvh, query=query, mode=mode, pc=pc,
                         rays=torch.from_numpy(rays).cuda()))
    return jobs


def _new_pred(hrpp, job):
    if job["pc"] is None:
        return None
    T, W, qo, qd, E = job["pc"][:5]
    hm, gu = (job["pc"][5], job["pc"][6]) if len(job["pc"]) > 5 else (0, 0)
    il, rp = (job["pc"][7], job["pc"][8]) if len(job["pc"]) > 7 else (0, 0)
    fe = job["pc"][9] if len(job["pc"]) > 9 else 0
    return hrpp.Predictor(job["bvh"], T, W, qo, qd, E, hash_mode=hm, go_up_level=gu, inline_lanes=il,
                          replace_policy=rp, first_epoch_rays=fe)


def _method_stats(hrpp, st):
    # the method's counters; the schedule counters (how fallback work was
    # split between kernels) may differ between a batch and a single call
    return {k: v for k, v in hrpp.stats_dict(st).items() if k not in hrpp.SCHEDULE_STATS}


def _single(hrpp, torch, job, pred):
    st = hrpp.new_stats()
    if job["query"] == "any":
        out = hrpp.trace_anyhit(job["bvh"], pred, job["rays"], stats=st)
    else:
        out = hrpp.trace_closest(job["bvh"], pred, job["rays"], mode=job["mode"], stats=st)
    torch.cuda.synchronize()
    return out.cpu().numpy().tobytes(), _method_stats(hrpp, st), (pred.export_raw().tobytes() if pred else b"")


def test_batch_equals_single_calls(hrpp):
    import torch
    _say("batch: building scenes")
    jobs = _build(hrpp, torch)
    ref = []
    for j in jobs:
        pred = _new_pred(hrpp, j)
        ref.append(_single(hrpp, torch, j, pred))
    # the oracle agrees with the single calls for every job: results, the
    # method's counters and (with a predictor) the table's tags and slots
    for k, j in enumerate(jobs):
        _say(f"batch: oracle for job {k}")
        ob = oracle.build_sah(j["tris"])
        if j["pc"] is None:
            want, ws = oracle.trace(ob, j["tris"], j["rays_np"], query=j["query"], mode=j["mode"])
            got_table = None
        else:
            T, W, qo, qd, E = j["pc"][:5]
            hm, gu = (j["pc"][5], j["pc"][6]) if len(j["pc"]) > 5 else (0, 0)
            rp = j["pc"][8] if len(j["pc"]) > 8 else 0
            fe = j["pc"][9] if len(j["pc"]) > 9 else 0
            tb = oracle.Table(T, W, qo, qd, hash_mode=hm, go_up=gu, policy=rp)
            want, ws = oracle.trace(ob, j["tris"], j["rays_np"], query=j["query"], mode=j["mode"], table=tb,
                                    epoch=E, first_epoch=fe)
            got_table = tb
        assert want.tobytes() == ref[k][0], f"job {k}: results differ from the oracle"
        assert {n: v for n, v in ref[k][1].items() if n in ws} == ws, f"job {k}: counters differ from the oracle"
        if got_table is not None:
            raw = np.frombuffer(ref[k][2], np.uint8).reshape(1 << got_table.log2n, -1)
            assert np.array_equal(raw[:, :8].copy().view(np.uint64)[:, 0], got_table.tags), f"job {k}: tags"
            W = got_table.W
            assert np.array_equal(raw[:, 8:8 + 4 * W].copy().view(np.uint32), got_table.slots), f"job {k}: slots"
    for use_graph in (False, True):
        _say(f"batch: graph={use_graph}")
        preds = [_new_pred(hrpp, j) for j in jobs]
        stats = [hrpp.new_stats() for _ in jobs]
        b = hrpp.Batch([dict(bvh=j["bvh"], pred=p, rays=j["rays"], query=j["query"], mode=j["mode"], stats=s)
                        for j, p, s in zip(jobs, preds, stats)])
        replays = 3 if use_graph else 1
        for rep in range(replays):
            for p in preds:
                if p is not None:
                    p.reset()
            for s in stats:
                s.zero_()
            torch.cuda.synchronize()
            b.launch(use_graph=use_graph)
            torch.cuda.synchronize()
            hrpp.get_error()
            for k, j in enumerate(jobs):
                got = (b.outputs[k].cpu().numpy().tobytes(), _method_stats(hrpp, stats[k]),
                       preds[k].export_raw().tobytes() if preds[k] else b"")
                assert got[0] == ref[k][0], f"job {k} results differ (graph={use_graph}, replay {rep})"
                assert got[1] == ref[k][1], f"job {k} counters differ (graph={use_graph}, replay {rep})"
                assert got[2] == ref[k][2], f"job {k} table differs (graph={use_graph}, replay {rep})"
            # eager work between replays
            _ = _single(hrpp, torch, jobs[0], None)
        b.close()


def test_batch_rejects_shared_predictor(hrpp):
    import torch
    tris = sg.soup_scene(5, 500)
    bvh = hrpp.BVH(tris)
    p = hrpp.Predictor(bvh, 10, 4, 4, 4, 256)
    r = torch.from_numpy(sg.tiny_shadow_rays(5, 300)).cuda()
    with pytest.raises(hrpp.HrppError):
        hrpp.Batch([dict(bvh=bvh, pred=p, rays=r), dict(bvh=bvh, pred=p, rays=r)])


def test_batch_many_jobs_per_group(hrpp):
    # 140 predictor jobs in one group and 70 plain ones: each launch's flat
    # grid finds a block's job among more than 64 offsets (several wave-wide
    # rounds), so jobs past the first 64 are placed correctly; every job is
    # checked against the oracle
    import torch
    _say("batch: many jobs per group")
    scenes = []
    for s in range(5):
        tris = sg.mixed_scene(40 + s, 300 + 400 * s)
        scenes.append((tris, hrpp.BVH(tris), oracle.build_sah(tris)))
    rng = np.random.default_rng(7)
    jobs, specs = [], []
    for k in range(210):
        tris, bvh, ob = scenes[k % len(scenes)]
        n = int(rng.integers(1, 3000))
        sh, ao = sg.secondary_rays_on_surface(tris, n, 500 + k)
        rays = np.ascontiguousarray(np.concatenate([sh, ao]))
        pc = None if k >= 140 else (int(rng.integers(6, 12)), 4, 5, 6, int(rng.integers(64, 1024)))
        specs.append((tris, ob, rays, pc))
        jobs.append(dict(bvh=bvh, rays=torch.from_numpy(rays).cuda(), query="any"))
    for use_graph in (False, True):
        preds = [hrpp.Predictor(j["bvh"], *pc) if pc else None for j, (_, _, _, pc) in zip(jobs, specs)]
        stats = [hrpp.new_stats() for _ in jobs]
        b = hrpp.Batch([dict(j, pred=p, stats=s) for j, p, s in zip(jobs, preds, stats)])
        torch.cuda.synchronize()
        b.launch(use_graph=use_graph)
        torch.cuda.synchronize()
        hrpp.get_error()
        for k, (tris, ob, rays, pc) in enumerate(specs):
            tb = oracle.Table(*pc[:4]) if pc else None
            want, ws = oracle.trace(ob, tris, rays, query="any", table=tb, epoch=pc[4] if pc else 1 << 30)
            assert b.outputs[k].cpu().numpy().tobytes() == want.tobytes(), f"job {k}: results (graph={use_graph})"
            got = _method_stats(hrpp, stats[k])
            assert {n: v for n, v in got.items() if n in ws} == ws, f"job {k}: counters (graph={use_graph})"
            if pc:
                tags, slots = preds[k].export()
                assert np.array_equal(tags, tb.tags) and np.array_equal(slots, tb.slots), f"job {k}: table"
        b.close()
