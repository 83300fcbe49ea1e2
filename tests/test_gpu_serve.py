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
    # the oracle agrees for two requests
    for i in range(2):
        r = reqs[i]
        sc = scenes[r["scene"]]
        want, _ = oracle.trace(oracle.build_sah(sc["tris"]), sc["tris"], r["rays"].numpy(), query=r["query"],
                               mode="exact")
        assert want.tobytes() == alone[i]
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
    srv.close()
