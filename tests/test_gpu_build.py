"""GPU parity of the device BVH build.

The linear BVH the library builds on the GPU must equal the oracle's linear
BVH node for node: box bit patterns, right children, leaf ranges, depths and
the triangle order.  Queries traced over it must equal the oracle's traces
over the same tree (results, every counter, table bytes), and any-hit flags
and exact closest hits must equal those over the host SAH tree, since they
do not depend on the tree.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import scenegen as sg
from tests.test_gpu_parity import check_case, device_bvh

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


def _dev(tris):
    import torch
    return torch.from_numpy(np.ascontiguousarray(tris, np.float32)).cuda()


@pytest.mark.parametrize("n,leaf_max", [(1, 4), (3, 4), (4, 4), (5, 4), (64, 1), (257, 2), (3000, 4), (3000, 8),
                                        (4097, 3), (70001, 4),
                                        # the sort's sub-tiles of 1,024 items and the prefix sum's
                                        # tiles of 4,096 words (n + 1 of them): sizes at both edges
                                        (1023, 2), (1024, 2), (1025, 2), (2048, 1), (2049, 2), (4094, 2),
                                        (4095, 2), (4096, 2), (8191, 2), (8193, 2), (263169, 2)])
def test_device_build_equals_oracle(hrpp, n, leaf_max):
    _say(f"device build soup n={n} leaf_max={leaf_max}")
    tris = sg.triangle_soup(70 + n, n)
    if n >= 3000:
        tris[: n // 3] = tris[n // 3: 2 * (n // 3)]         # many equal codes
    bvh, ob = device_bvh(hrpp, tris, leaf_max)
    oracle.validate_bvh(ob, tris, leaf_max, 64)


@pytest.mark.parametrize("n,leaf_max,passes", [(2, 1, 1), (3, 1, 1), (7, 1, 1), (8, 1, 3), (64, 1, 2), (257, 2, 1),
                                               (3000, 4, 2), (4097, 3, 1), (70001, 2, 2), (263169, 2, 1)])
def test_device_treelet_build_equals_oracle(hrpp, n, leaf_max, passes):
    _say(f"device treelet build soup n={n} leaf_max={leaf_max} passes={passes}")
    tris = sg.triangle_soup(170 + n, n)
    if n >= 3000:
        tris[: n // 3] = tris[n // 3: 2 * (n // 3)]         # many equal codes
    bvh, ob = device_bvh(hrpp, tris, leaf_max, passes=passes)
    oracle.validate_bvh(ob, tris, leaf_max, 64)


def test_device_treelet_build_scenes(hrpp):
    _say("device treelet build: heightfield 2^20, degenerate scenes")
    device_bvh(hrpp, sg.heightfield_scene(93, 1 << 20), 2, passes=2)
    device_bvh(hrpp, np.repeat(sg.triangle_soup(5, 1), 50, axis=0), 1, passes=2)
    signed = sg.triangle_soup(7, 300) - 0.5
    signed[::7, 0, 0] = 0.0
    signed[1::7, 1, 0] = -0.0
    signed[2::7, :, 2] = -0.0
    device_bvh(hrpp, signed, 2, passes=3)
    device_bvh(hrpp, np.zeros((9, 9), np.float32), 2, passes=1)


def test_device_treelet_depth_limit(hrpp):
    # with treelet passes max_depth bounds the restructured tree, not the
    # linear BVH before them: here the passes make the tree one level
    # shallower, so the limit of the restructured depth builds while the
    # linear BVH alone would not, and one level less reports EDEPTH, on both
    # sides
    tris = sg.triangle_soup(211, 3000)
    deep = oracle.build_lbvh(tris, leaf_max=1, treelet_passes=2).max_depth()
    base = oracle.build_lbvh(tris, leaf_max=1).max_depth()
    _say(f"device treelet depth limit: linear {base}, restructured {deep}")
    assert deep < base
    with pytest.raises(hrpp.HrppError, match="deeper"):
        hrpp.BVH.build_on_device(_dev(tris), leaf_max=1, max_depth=deep)
    device_bvh(hrpp, tris, 1, max_depth=deep, passes=2)
    with pytest.raises(ValueError):
        oracle.build_lbvh(tris, leaf_max=1, max_depth=deep - 1, treelet_passes=2)
    with pytest.raises(hrpp.HrppError, match="deeper"):
        hrpp.BVH.build_on_device(_dev(tris), leaf_max=1, max_depth=deep - 1, treelet_passes=2)


def test_device_build_large(hrpp):
    # 2^22 triangles (a heightfield), and 2^20 copies of one triangle, where
    # every split falls back to the positions' bits
    _say("device build 2^22 heightfield")
    device_bvh(hrpp, sg.heightfield_scene(91, 1 << 22), 4)
    _say("device build 2^20 equal triangles")
    bvh, ob = device_bvh(hrpp, np.repeat(sg.triangle_soup(92, 1), 1 << 20, axis=0), 2)
    assert bvh.max_depth == 19                  # a balanced tree: 2^19 leaves of two


def test_device_build_degenerate_scenes(hrpp):
    _say("device build degenerate scenes")
    same = np.repeat(sg.triangle_soup(5, 1), 50, axis=0)    # one code: splits by position
    device_bvh(hrpp, same, 1)
    flat = sg.triangle_soup(6, 500)
    flat[:, :, 1] = 0.25                                    # a flat axis: one cell
    device_bvh(hrpp, flat, 4)
    signed = sg.triangle_soup(7, 300) - 0.5                 # coordinates of both signs and of both zeros
    signed[::7, 0, 0] = 0.0
    signed[1::7, 1, 0] = -0.0
    signed[2::7, :, 2] = -0.0
    device_bvh(hrpp, signed, 2)
    point = np.zeros((9, 9), np.float32)                    # every triangle a point at the origin
    device_bvh(hrpp, point, 2)


def test_device_build_errors(hrpp):
    import torch
    _say("device build errors")
    same = np.repeat(sg.triangle_soup(5, 1), 50, axis=0)
    with pytest.raises(hrpp.HrppError, match="deeper"):
        hrpp.BVH.build_on_device(_dev(same), leaf_max=1, max_depth=3)
    bad = sg.triangle_soup(8, 100)
    bad[37, 1, 2] = np.nan
    with pytest.raises(hrpp.HrppError, match="invalid"):
        hrpp.BVH.build_on_device(_dev(bad))
    bad[37, 1, 2] = np.inf
    with pytest.raises(hrpp.HrppError, match="invalid"):
        hrpp.BVH.build_on_device(_dev(bad))
    with pytest.raises(hrpp.HrppError, match="invalid"):
        hrpp.BVH.build_on_device(_dev(sg.triangle_soup(8, 10)), leaf_max=9)
    bvh = hrpp.BVH.build_on_device(_dev(sg.triangle_soup(8, 100)))
    rays = torch.from_numpy(sg.tiny_shadow_rays(8, 64)).cuda()
    with pytest.raises(hrpp.HrppError):
        hrpp.trace_wide_anyhit(bvh, rays)
    with pytest.raises(hrpp.HrppError):
        bvh.upload()
    # the library rejects a scratch or BVH buffer that is too small, without launching
    lib = hrpp.load_library()
    import ctypes as C
    v = _dev(sg.triangle_soup(8, 100))
    desc = hrpp.hrpp._BvhDesc(4, 32, 64)
    need = lib.hrpp_bvh_device_build_scratch_bytes(100)
    size = lib.hrpp_bvh_required_bytes(100, C.byref(desc))
    raw, buf = hrpp.hrpp._aligned(size, "cuda")
    sraw, scr = hrpp.hrpp._aligned(need, "cuda")
    h = C.c_void_p()
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.hrpp_build_bvh_device(v.data_ptr(), 100, C.byref(desc), scr.data_ptr(), need - 1, buf.data_ptr(),
                                     size, s, C.byref(h)) == 2
    assert lib.hrpp_build_bvh_device(v.data_ptr(), 100, C.byref(desc), scr.data_ptr(), need, buf.data_ptr(),
                                     size - 256, s, C.byref(h)) == 2
    assert lib.hrpp_build_bvh_device(v.data_ptr(), 100, C.byref(desc), scr.data_ptr() + 4, need, buf.data_ptr(),
                                     size, s, C.byref(h)) == 1
    assert not h.value


def test_device_build_reuses_scratch(hrpp):
    # two builds in a row through one scratch buffer, the second smaller
    import ctypes as C
    import torch
    _say("device build scratch reuse")
    lib = hrpp.load_library()
    desc = hrpp.hrpp._BvhDesc(4, 32, 64)
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    need = lib.hrpp_bvh_device_build_scratch_bytes(20000)
    sraw, scr = hrpp.hrpp._aligned(need, "cuda")
    for n, seed in ((20000, 81), (777, 82)):
        tris = sg.triangle_soup(seed, n)
        size = lib.hrpp_bvh_required_bytes(n, C.byref(desc))
        raw, buf = hrpp.hrpp._aligned(size, "cuda")
        h = C.c_void_p()
        v = _dev(tris)
        assert lib.hrpp_build_bvh_device(v.data_ptr(), n, C.byref(desc), scr.data_ptr(), need, buf.data_ptr(), size,
                                         s, C.byref(h)) == 0
        b = hrpp.BVH.__new__(hrpp.BVH)
        b.handle, b.num_tris, b.buffer = h, n, buf
        nn = C.c_uint32()
        lib.hrpp_bvh_info(h, C.byref(nn), None, None)
        b.num_nodes = nn.value
        got = b.export()
        ob = oracle.build_lbvh(tris)
        assert np.array_equal(got["box"].view(np.uint32), ob.box.view(np.uint32))
        assert np.array_equal(got["right"], ob.right) and np.array_equal(got["perm"], ob.perm)
        b.close()


def test_device_tree_tiny_queries(hrpp):
    tris, rays = sg.tiny_workload()
    check_case(hrpp, "tiny plain (device tree)", tris, rays, builder="device")
    check_case(hrpp, "tiny hrpp (device tree)", tris, rays, pred_cfg=(12, 4, 5, 6, 256), builder="device", calls=2)
    check_case(hrpp, "tiny closest paper (device tree)", tris, rays, query="closest", mode="paper",
               pred_cfg=(12, 4, 5, 6, 256), builder="device")
    check_case(hrpp, "tiny go-up 2 (device tree)", tris, rays, pred_cfg=(12, 4, 5, 6, 256, 0, 2), builder="device")


@pytest.fixture(scope="module")
def small_terrain():
    return sg.terrain_workload(total=30000, width=320, height=180)


def test_device_tree_terrain_queries(hrpp, small_terrain):
    tris, prim = small_terrain
    check_case(hrpp, "terrain primary paper (device tree)", tris, prim, query="closest", mode="paper",
               pred_cfg=(16, 8, 5, 7, 4096, 0, 0, 0, 0, 1024), builder="device")
    he, _ = oracle.trace(oracle.build_sah(tris), tris, prim, query="closest", mode="exact")
    got, _ = check_case(hrpp, "terrain primary exact (device tree)", tris, prim, query="closest", mode="exact",
                        builder="device")
    assert got.tobytes() == he.tobytes()                    # the same hits as over the SAH tree
    shadow = sg.shadow_rays_from_hits(tris, prim, he[:, 0], he[:, 3].view(np.uint32), seed=5)
    occ_sah, _ = oracle.trace(oracle.build_sah(tris), tris, shadow)
    got, _ = check_case(hrpp, "terrain shadow hrpp go-up 1 (device tree)", tris, shadow,
                        pred_cfg=(16, 8, 6, 3, 8192, 0, 1), builder="device")
    assert np.array_equal(got, occ_sah)


def test_treelet_tree_queries(hrpp, small_terrain):
    # traces over the restructured device tree: leaves at new positions,
    # predicted subtrees named by the new canonical numbering
    tris, rays = sg.tiny_workload()
    check_case(hrpp, "tiny hrpp (treelet tree)", tris, rays, pred_cfg=(12, 4, 5, 6, 256), builder="device",
               passes=2, calls=2)
    check_case(hrpp, "tiny closest exact go-up 2 (treelet tree)", tris, rays, query="closest", mode="exact",
               pred_cfg=(12, 4, 5, 6, 256, 0, 2), builder="device", passes=2)
    tris, prim = small_terrain
    check_case(hrpp, "terrain primary paper (treelet tree)", tris, prim, query="closest", mode="paper",
               pred_cfg=(16, 8, 5, 7, 4096, 0, 0, 0, 0, 1024), builder="device", passes=2, leaf_max=2)
    he, _ = oracle.trace(oracle.build_sah(tris), tris, prim, query="closest", mode="exact")
    got, _ = check_case(hrpp, "terrain primary exact go-up 1 (treelet tree)", tris, prim, query="closest",
                        mode="exact", pred_cfg=(14, 8, 5, 7, 4096, 0, 1), builder="device", passes=1)
    assert got.tobytes() == he.tobytes()
    shadow = sg.shadow_rays_from_hits(tris, prim, he[:, 0], he[:, 3].view(np.uint32), seed=5)
    check_case(hrpp, "terrain shadow go-up 1 (treelet tree)", tris, shadow, pred_cfg=(16, 8, 6, 3, 8192, 0, 1),
               builder="device", passes=2, leaf_max=2)


@pytest.fixture(scope="module")
def full_terrain():
    return sg.terrain_workload()


def test_device_tree_full_size(hrpp, full_terrain):
    # the at-scale scene (2^20 triangles) and its 2,073,600 primaries and
    # shadow rays, with the benchmark's leaf size and predictor configurations
    w = sg.AT_SCALE
    tris, prim = full_terrain
    pq, sq = w["primary_q"], w["shadow_q"]
    cfg_all = (w["log2_entries"], w["ways"], pq[0], pq[1], pq[2], 0, 0, pq[3], 0, pq[4])
    cfg_any = (w["log2_entries"], w["ways"], sq[0], sq[1], sq[2], 0, 0, sq[3], 0, sq[4])
    _, st = check_case(hrpp, "full primary paper (device tree)", tris, prim, query="closest", mode="paper",
                       pred_cfg=cfg_all, builder="device", leaf_max=w["leaf_max"])
    assert st["rays"] == 1920 * 1080
    he, _ = oracle.trace(oracle.build_sah(tris), tris, prim, query="closest", mode="exact")
    shadow = sg.shadow_rays_from_hits(tris, prim, he[:, 0], he[:, 3].view(np.uint32), seed=w["seed"],
                                      light_center=w["light_center"], light_size=w["light_size"])
    check_case(hrpp, "full shadow hrpp (device tree)", tris, shadow, pred_cfg=cfg_any, builder="device",
               leaf_max=w["leaf_max"])
    check_case(hrpp, "full shadow plain (device tree, leaves of 4)", tris, shadow, builder="device")


def test_serving_device_built_scenes(hrpp):
    # scenes built on the device serve requests like host-built ones, also a
    # scene added while the server runs: any-hit flags and exact closest hits
    # equal the oracle's
    import torch
    _say("serving device-built scenes")
    scenes = []
    for k in range(3):
        tris = sg.mixed_scene(930 + k, [30000, 8000, 20000][k])
        bvh = hrpp.BVH.build_on_device(_dev(tris)) if k != 2 else None
        sh, ao = sg.secondary_rays_on_surface(tris, 20000, 960 + k)
        prim = sh.copy()
        prim[:, 7] = np.inf
        scenes.append(dict(tris=tris, bvh=bvh, sec=np.concatenate([sh, ao]), prim=prim))
    for sc in scenes[:2]:
        sc["anyp"] = [hrpp.Predictor(sc["bvh"], 14, 8, 5, 6, 4096)]
        sc["clp"] = [hrpp.Predictor(sc["bvh"], 14, 8, 5, 6, 4096)]
    srv = hrpp.Server([(s["bvh"], s["anyp"], s["clp"]) for s in scenes[:2]], slots=2, pool_bytes=8 << 20)

    def request(k, i, index=None):
        # rays of scenes[k], submitted to server scene `index` (default k)
        query = "any" if i % 3 else "closest"
        pool = scenes[k]["prim"] if query == "closest" else scenes[k]["sec"]
        rays = torch.from_numpy(np.ascontiguousarray(pool[i * 1000:(i + 1) * 1000 + 4000])).pin_memory()
        n = rays.shape[0]
        out = (torch.empty(n, dtype=torch.uint8) if query == "any" else
               torch.empty((n, 4), dtype=torch.float32)).pin_memory()
        return dict(scene=k, query=query, rays=rays, out=out,
                    id=srv.submit(k if index is None else index, query, rays, out))

    reqs = [request(i % 2, i) for i in range(8)]
    # a third scene arrives while those run: built on the device, then added
    sc = scenes[2]
    sc["bvh"] = hrpp.BVH.build_on_device(_dev(sc["tris"]))
    sc["anyp"] = [hrpp.Predictor(sc["bvh"], 12, 4, 5, 6, 2048)]
    sc["clp"] = [hrpp.Predictor(sc["bvh"], 12, 4, 5, 6, 2048)]
    with pytest.raises(hrpp.HrppError):          # a predictor that serves scene 0 (and indexes its tree)
        srv.add_scene(sc["bvh"], scenes[0]["anyp"], sc["clp"])
    with pytest.raises(hrpp.HrppError):          # no scene 2 yet
        srv.submit(2, "any", reqs[0]["rays"], reqs[0]["out"])
    assert srv.add_scene(sc["bvh"], sc["anyp"], sc["clp"]) == 2
    reqs += [request(2, i) for i in range(6)] + [request(0, 9)]
    # scene 1 leaves while its requests may still run: the call waits for them
    srv.remove_scene(1)
    retired = set()
    for r in reqs:
        if r["scene"] == 1:
            assert srv.poll(r["id"])["state"] == 2   # this final poll retires the request
            retired.add(r["id"])
    with pytest.raises(hrpp.HrppError):          # no new requests for a removed scene
        srv.submit(1, "any", reqs[0]["rays"], reqs[0]["out"])
    with pytest.raises(hrpp.HrppError):          # removed already
        srv.remove_scene(1)
    # its predictors may serve again, with another scene on the same tree
    assert srv.add_scene(scenes[1]["bvh"], scenes[1]["anyp"], scenes[1]["clp"]) == 3
    reqs += [request(1, 2, index=3), request(1, 4, index=3)]
    srv.wait_all()
    for r in reqs:
        sc = scenes[r["scene"]]
        if r["id"] not in retired:
            assert srv.poll(r["id"])["state"] == 2
        want, _ = oracle.trace(oracle.build_sah(sc["tris"]), sc["tris"], r["rays"].numpy(), query=r["query"],
                               mode="exact")
        assert r["out"].numpy().tobytes() == want.tobytes()
    srv.close()


def test_batch_over_device_built_scenes(hrpp):
    # a graph-captured batch over device-built scenes computes what each job's
    # own call computes, on every replay; one job also against the oracle
    import torch
    from tests.test_gpu_batch import _jobs_spec, _method_stats, _new_pred, _single
    _say("batch over device-built scenes")
    jobs = []
    for seed, ntri, nray, query, mode, pc in [j for k, j in enumerate(_jobs_spec()) if k in (0, 2, 3, 4, 9, 13)]:
        tris = sg.mixed_scene(seed, ntri)
        sh, ao = sg.secondary_rays_on_surface(tris, nray, seed + 100)
        rays = np.concatenate([sh, ao])
        if query == "closest":
            rays[:, 7] = np.inf
        jobs.append(dict(tris=tris, rays_np=rays, bvh=hrpp.BVH.build_on_device(_dev(tris)), query=query, mode=mode,
                         pc=pc, rays=torch.from_numpy(rays).cuda()))
    ref = [_single(hrpp, torch, j, _new_pred(hrpp, j)) for j in jobs]
    j = jobs[0]
    T, W, qo, qd, E = j["pc"][:5]
    want, ws = oracle.trace(oracle.build_lbvh(j["tris"]), j["tris"], j["rays_np"], query=j["query"], mode=j["mode"],
                            table=oracle.Table(T, W, qo, qd), epoch=E)
    assert want.tobytes() == ref[0][0] and ws == ref[0][1]
    preds = [_new_pred(hrpp, j) for j in jobs]
    stats = [hrpp.new_stats() for _ in jobs]
    b = hrpp.Batch([dict(bvh=j["bvh"], pred=p, rays=j["rays"], query=j["query"], mode=j["mode"], stats=s)
                    for j, p, s in zip(jobs, preds, stats)])
    for rep in range(3):
        for p in preds:
            if p is not None:
                p.reset()
        for s in stats:
            s.zero_()
        torch.cuda.synchronize()
        b.launch(use_graph=True)
        torch.cuda.synchronize()
        for k in range(len(jobs)):
            assert b.outputs[k].cpu().numpy().tobytes() == ref[k][0], f"job {k} results differ (replay {rep})"
            assert _method_stats(hrpp, stats[k]) == ref[k][1], f"job {k} counters differ (replay {rep})"
            assert (preds[k].export_raw().tobytes() if preds[k] else b"") == ref[k][2], f"job {k} table (replay {rep})"
        _ = _single(hrpp, torch, jobs[0], None)
    b.close()
