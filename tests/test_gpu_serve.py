"""Serving: every request's results are the same alone and in the mix, the
device pool (HBM budget) is never exceeded, and oversize requests are refused."""
from __future__ import annotations

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


def test_requests_same_alone_and_in_mix(hrpp):
    import torch
    print("[gpu-case] serving mix", flush=True)
    g = np.random.default_rng(9)
    scenes = []
    for k in range(3):
        tris = sg.mixed_scene(900 + k, [20000, 5000, 40000][k])
        bvh = hrpp.BVH(tris)
        anyp = [hrpp.Predictor(bvh, 14, 8, 5, 6, 4096) for _ in range(2)]
        clp = [hrpp.Predictor(bvh, 14, 8, 5, 6, 4096)]
        sh, ao = sg.secondary_rays_on_surface(tris, 60000, 950 + k)
        prim = sh.copy()
        prim[:, 7] = np.inf
        scenes.append(dict(tris=tris, bvh=bvh, anyp=anyp, clp=clp, sec=np.concatenate([sh, ao]), prim=prim))
    reqs = []
    for i in range(48):
        k = int(g.integers(0, 3))
        query = "closest" if g.random() < 0.3 else "any"
        n = int(g.integers(1000, 40000))
        pool = scenes[k]["prim"] if query == "closest" else scenes[k]["sec"]
        off = int(g.integers(0, pool.shape[0] - n))
        rays = torch.from_numpy(np.ascontiguousarray(pool[off:off + n])).pin_memory()
        out = (torch.empty(n, dtype=torch.uint8) if query == "any" else torch.empty((n, 4), dtype=torch.float32)).pin_memory()
        reqs.append(dict(scene=k, query=query, rays=rays, out=out))
    # alone: plain traversal of each request, one at a time
    alone = []
    for r in reqs:
        sc = scenes[r["scene"]]
        rd = r["rays"].cuda()
        o = hrpp.trace_anyhit(sc["bvh"], None, rd) if r["query"] == "any" else \
            hrpp.trace_closest(sc["bvh"], None, rd, mode="exact")
        alone.append(o.cpu().numpy().tobytes())
    # the oracle agrees for every request (plain traversal; the results of
    # both served queries do not depend on the tables)
    obvh = [oracle.build_sah(sc["tris"]) for sc in scenes]
    for i, r in enumerate(reqs):
        sc = scenes[r["scene"]]
        want, _ = oracle.trace(obvh[r["scene"]], sc["tris"], r["rays"].numpy(), query=r["query"], mode="exact")
        assert want.tobytes() == alone[i], f"request {i} differs from the oracle"
    # in the mix: all at once through a small pool that forces queueing
    pool_bytes = 3 << 20
    srv = hrpp.Server([(s["bvh"], s["anyp"], s["clp"]) for s in scenes], slots=4, pool_bytes=pool_bytes)
    for rep in range(2):           # the second pass runs with warm tables
        ids = [srv.submit(r["scene"], r["query"], r["rays"], r["out"]) for r in reqs]
        srv.wait_all()
        for i, (r, rid) in enumerate(zip(reqs, ids)):
            info = srv.poll(rid)
            assert info["state"] == 2 and info["status"] == 0
            assert info["latency_ms"] >= info["service_ms"] >= 0
            assert r["out"].numpy().tobytes() == alone[i], f"request {i} differs in the mix (pass {rep})"
    assert 0 < srv.pool_peak() <= pool_bytes
    big = torch.zeros((200000, 8), dtype=torch.float32).pin_memory()
    with pytest.raises(hrpp.HrppError):
        srv.submit(0, "any", big, torch.empty(200000, dtype=torch.uint8).pin_memory())
    # every request was retired by its final poll
    assert srv.held() == 0
    with pytest.raises(hrpp.HrppError):
        srv.poll(ids[0])
    srv.close()


def test_long_run_holds_bounded_records(hrpp):
    # 20,000 small requests, each polled until done: the server's request
    # records stay bounded by what is in flight, not by what was ever submitted
    import torch
    print("[gpu-case] serving 20000 small requests", flush=True)
    tris = sg.mixed_scene(990, 3000)
    bvh = hrpp.BVH(tris)
    anyp = [hrpp.Predictor(bvh, 12, 4, 5, 6, 1024) for _ in range(2)]
    clp = [hrpp.Predictor(bvh, 12, 4, 5, 6, 1024)]
    sh, _ = sg.secondary_rays_on_surface(tris, 4096, 991)
    rays = torch.from_numpy(np.ascontiguousarray(sh[:64])).pin_memory()
    ob = oracle.build_sah(tris)
    want, _ = oracle.trace(ob, tris, sh[:64], query="any", mode="exact")
    srv = hrpp.Server([(bvh, anyp, clp)], slots=4, pool_bytes=1 << 20)
    window, live, peak_held = 64, [], 0
    outs = [torch.empty(64, dtype=torch.uint8).pin_memory() for _ in range(window)]
    for i in range(20000):
        if len(live) == window:                  # keep at most `window` requests in flight
            rid, o = live.pop(0)
            while srv.poll(rid)["state"] != 2:
                pass
            assert o.numpy().tobytes() == want.tobytes()
        o = outs[i % window]
        live.append((srv.submit(0, "any", rays, o), o))
        if i % 1000 == 0:
            peak_held = max(peak_held, srv.held())
    for rid, o in live:
        while srv.poll(rid)["state"] != 2:
            pass
        assert o.numpy().tobytes() == want.tobytes()
    srv.wait_all()
    assert peak_held <= window and srv.held() == 0
    srv.close()
