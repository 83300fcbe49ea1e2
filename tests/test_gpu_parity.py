"""GPU parity: the HIP library against the CPU oracle, element by element.

Any-hit flags, closest hits (t, u, v, prim bit patterns), every counter and
the predictor table bytes must match exactly; both sides run the same
binary32 operation sequence.  (The stated tolerance for floating-point
outputs -- t within 1e-5 relative, barycentrics within 1e-5 absolute -- is
therefore met with zero error; a mismatch beyond it fails as well.)
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
import scenegen as sg

pytestmark = pytest.mark.gpu

NONE32 = 0xFFFFFFFF


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


def gpu_run(hrpp, bvh, rays, query="any", mode="paper", pred=None, stats=None):
    import torch
    r = torch.from_numpy(np.ascontiguousarray(rays, np.float32)).cuda()
    st = stats if stats is not None else hrpp.new_stats()
    if query == "any":
        out = hrpp.trace_anyhit(bvh, pred, r, stats=st)
    else:
        out = hrpp.trace_closest(bvh, pred, r, mode=mode, stats=st)
    torch.cuda.synchronize()
    hrpp.get_error(bvh)
    return out.cpu().numpy(), hrpp.stats_dict(st)


def assert_same_result(query, got, want):
    if query == "any":
        assert got.dtype == np.uint8
        bad = np.nonzero(got != want)[0]
        assert bad.size == 0, f"{bad.size} flags differ, first rays {bad[:8]}"
    else:
        g, w = got.view(np.uint32), want.view(np.uint32)
        bad = np.nonzero(np.any(g != w, axis=1))[0]
        if bad.size:
            i = bad[0]
            raise AssertionError(f"{bad.size} hits differ; ray {i}: gpu {got[i]} {g[i, 3]} oracle {want[i]} {w[i, 3]}")


def assert_same_table(pred, tb: oracle.Table):
    tags, slots = pred.export()
    assert np.array_equal(tags, tb.tags), f"{int(np.count_nonzero(tags != tb.tags))} tags differ"
    assert np.array_equal(slots, tb.slots), f"{int(np.count_nonzero(np.any(slots != tb.slots, 1)))} entries differ"


def device_bvh(hrpp, tris, leaf_max=4, max_depth=64, passes=0):
    """The library's device-built linear BVH (after `passes` treelet passes),
    checked against the oracle's."""
    import torch
    bvh = hrpp.BVH.build_on_device(torch.from_numpy(np.ascontiguousarray(tris, np.float32)).cuda(),
                                   leaf_max=leaf_max, max_depth=max_depth, treelet_passes=passes)
    ob = oracle.build_lbvh(tris, leaf_max=leaf_max, max_depth=max_depth, treelet_passes=passes)
    got = bvh.export()
    assert bvh.num_nodes == ob.num_nodes
    assert np.array_equal(got["box"].view(np.uint32), ob.box.view(np.uint32)), "boxes differ"
    for k in ("right", "first", "count", "depth", "perm"):
        assert np.array_equal(got[k], getattr(ob, k)), f"{k} differs"
    assert bvh.max_depth == ob.max_depth()
    return bvh, ob


def check_case(hrpp, name, tris, rays, query="any", mode="paper", pred_cfg=None, calls=1, leaf_max=4,
               builder="sah", passes=0):
    """Run `calls` successive traces of `rays` on both sides and compare all.

    builder "sah": the host SAH tree on both sides; "device": the library's
    device-built linear BVH against the oracle's; either after `passes`
    treelet passes."""
    _say(f"{name}: {tris.shape[0]} tris, {rays.shape[0]} rays, {query}/{mode}, pred={pred_cfg}, calls={calls}, "
         f"builder={builder}, passes={passes}")
    if builder == "device":
        bvh, ob = device_bvh(hrpp, tris, leaf_max, passes=passes)
    else:
        bvh = hrpp.BVH(tris, leaf_max=leaf_max, treelet_passes=passes)
        ob = oracle.build_sah(tris, leaf_max=leaf_max, treelet_passes=passes)
    vtx = oracle.bvh_vertices(tris, ob)
    pred = tb = None
    if pred_cfg is not None:
        T, W, qo, qd, E = pred_cfg[:5]
        hm = pred_cfg[5] if len(pred_cfg) > 5 else 0
        gu = pred_cfg[6] if len(pred_cfg) > 6 else 0
        il = pred_cfg[7] if len(pred_cfg) > 7 else 0
        rp = pred_cfg[8] if len(pred_cfg) > 8 else 0
        fe = pred_cfg[9] if len(pred_cfg) > 9 else 0
        pred = hrpp.Predictor(bvh, log2_entries=T, ways=W, origin_bits=qo, dir_bits=qd, epoch_rays=E,
                              hash_mode=hm, go_up_level=gu, inline_lanes=il, replace_policy=rp, first_epoch_rays=fe)
        tb = oracle.Table(T, W, qo, qd, hash_mode=hm, go_up=gu, policy=rp)
    first = None
    if pred is not None and rays.shape[0] > 0:
        # the first epoch of a new predictor sees an empty table: the GPU runs it in
        # its own kernel, whose schedule counters equal the oracle's counts for
        # those rays alone
        e0 = min(fe or pred_cfg[4], rays.shape[0])
        _, w0 = oracle.trace(ob, tris, rays[:e0], query=query, mode=mode, table=oracle.Table(T, W, qo, qd,
                             hash_mode=hm, go_up=gu, policy=rp), epoch=pred_cfg[4], vtx=vtx)
        first = {"empty_rays": w0["rays"], "empty_lookups": w0["lookups"],
                 "empty_interior_visited": w0["interior_visited"], "empty_tri_tests": w0["tri_tests"],
                 "empty_records": w0["records"]}
    gst = hrpp.new_stats()
    for c in range(calls):
        got, gs = gpu_run(hrpp, bvh, rays, query, mode, pred, gst)
        want, ws = oracle.trace(ob, tris, rays, query=query, mode=mode, table=tb,
                                epoch=pred_cfg[4] if pred_cfg else 1 << 30, vtx=vtx,
                                first_epoch=fe if pred_cfg else 0)
        assert_same_result(query, got, want)
        if c == 0:
            acc = dict(ws)
        else:
            acc = {k: acc[k] + ws[k] for k in acc}
        # every counter the method defines (the schedule counters are not among them)
        assert {k: gs[k] for k in acc} == acc, {k: (gs[k], acc[k]) for k in acc if gs[k] != acc[k]}
        if pred is not None:
            assert_same_table(pred, tb)
            # schedule counters: the first epoch (later calls add none), and the
            # queue split of the other epochs' fallback traversals
            if first is not None:
                assert {k: gs[k] for k in first} == first, ({k: gs[k] for k in first}, first)
            later = gs["traversals"] - gs["empty_lookups"]
            if il == 65:
                assert gs["queue_traversals"] == later
            elif il == 1:
                assert gs["queue_traversals"] == 0
            assert 0 <= gs["queue_traversals"] <= later
    return got, gs


# ---------------------------------------------------------------------------
# Tiny workload: 256 triangles, 4,096 shadow rays
# ---------------------------------------------------------------------------

def test_tiny_plain_anyhit(hrpp):
    tris, rays = sg.tiny_workload()
    occ, st = check_case(hrpp, "tiny plain", tris, rays)
    assert st["hits"] > 400


@pytest.mark.parametrize("epoch", [256, 1, 4096, 1000, 5000])
def test_tiny_hrpp_anyhit(hrpp, epoch):
    tris, rays = sg.tiny_workload()
    check_case(hrpp, f"tiny hrpp E={epoch}", tris, rays, pred_cfg=(12, 4, 5, 6, epoch))


def test_tiny_hrpp_successive_calls_accumulate(hrpp):
    tris, rays = sg.tiny_workload()
    _, st = check_case(hrpp, "tiny hrpp x3", tris, rays, pred_cfg=(12, 4, 5, 6, 256), calls=3)
    assert st["pred_hits"] > 0


@pytest.mark.parametrize("first", [1, 100, 256, 999])
def test_tiny_first_epoch(hrpp, first):
    # a shorter first epoch in every call, epochs of 1000 after it (ragged tail)
    tris, rays = sg.tiny_workload()
    _, st = check_case(hrpp, f"tiny first epoch {first}", tris, rays, pred_cfg=(12, 4, 5, 6, 1000, 0, 0, 0, 0, first),
                       calls=2)
    closest = rays.copy()
    closest[:, 7] = np.inf
    for mode in ("paper", "exact"):
        check_case(hrpp, f"tiny closest {mode} first epoch {first}", tris, closest, query="closest", mode=mode,
                   pred_cfg=(12, 4, 5, 6, 1000, 0, 0, 1, 0, first))


@pytest.mark.parametrize("mode", ["paper", "exact"])
def test_tiny_closest(hrpp, mode):
    tris, rays = sg.tiny_workload()
    rays = rays.copy()
    rays[:, 7] = np.inf
    check_case(hrpp, f"tiny closest plain {mode}", tris, rays, query="closest", mode=mode)
    check_case(hrpp, f"tiny closest hrpp {mode}", tris, rays, query="closest", mode=mode,
               pred_cfg=(12, 4, 5, 6, 256), calls=2)


# ---------------------------------------------------------------------------
# Scaled terrain: several epochs, coherent primaries, shadow and AO rays
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def small_terrain():
    tris, prim = sg.terrain_workload(total=30000, width=320, height=180)
    return tris, prim


@pytest.mark.parametrize("mode", ["paper", "exact"])
def test_terrain_primary_closest(hrpp, small_terrain, mode):
    tris, prim = small_terrain
    _, st = check_case(hrpp, f"terrain primary {mode}", tris, prim, query="closest", mode=mode,
                       pred_cfg=(14, 8, 5, 6, 4096))
    assert st["pred_hits"] > 1000


def test_terrain_shadow_and_ao(hrpp, small_terrain):
    tris, prim = small_terrain
    ob = oracle.build_sah(tris)
    he, _ = oracle.trace(ob, tris, prim, query="closest", mode="exact")
    t, p = he[:, 0], he[:, 3].view(np.uint32)
    shadow = sg.shadow_rays_from_hits(tris, prim, t, p, seed=2)
    check_case(hrpp, "terrain shadow plain", tris, shadow)
    check_case(hrpp, "terrain shadow hrpp", tris, shadow, pred_cfg=(14, 8, 5, 6, 4096))
    ao = sg.ao_rays_from_hits(tris, prim[:4000], t[:4000], p[:4000], seed=3, samples=8,
                              tmax=0.05 * sg.scene_diagonal(tris))
    check_case(hrpp, "terrain ao plain", tris, ao)
    check_case(hrpp, "terrain ao hrpp", tris, ao, pred_cfg=(14, 8, 4, 4, 2048))


@pytest.mark.parametrize("cfg", [(1, 1, 2, 2, 512), (4, 2, 3, 3, 777), (10, 8, 7, 7, 64), (16, 3, 1, 1, 4096)])
def test_terrain_table_shapes(hrpp, small_terrain, cfg):
    # tiny tables (heavy collisions), one way (drops), odd epochs (ragged tails)
    tris, prim = small_terrain
    check_case(hrpp, f"terrain table {cfg}", tris, prim[:20000], query="closest", mode="paper", pred_cfg=cfg)
    check_case(hrpp, f"terrain table {cfg} exact", tris, prim[:20000], query="closest", mode="exact", pred_cfg=cfg)


# ---------------------------------------------------------------------------
# Plain-traversal baseline on the 4-wide tree: results equal the oracle's
# plain traversal (any-hit flags, exact closest hits); the per-ray counts
# (rays, invalid, hits, traversals) match, the visit counts are its own
# ---------------------------------------------------------------------------

def wide_case(hrpp, name, tris, rays, query="any", leaf_max=4, passes=0):
    import torch
    _say(f"{name}: wide {query}, {tris.shape[0]} tris, {rays.shape[0]} rays, treelet passes {passes}")
    bvh = hrpp.BVH(tris, leaf_max=leaf_max, treelet_passes=passes)
    ob = oracle.build_sah(tris, leaf_max=leaf_max, treelet_passes=passes)
    vtx = oracle.bvh_vertices(tris, ob)
    r = torch.from_numpy(np.ascontiguousarray(rays)).cuda()
    st = hrpp.new_stats()
    if query == "any":
        got = hrpp.trace_wide_anyhit(bvh, r, stats=st)
        want, ws = oracle.trace(ob, tris, rays, query="any", vtx=vtx)
    else:
        got = hrpp.trace_wide_closest(bvh, r, stats=st)
        want, ws = oracle.trace(ob, tris, rays, query="closest", mode="exact", vtx=vtx)
    torch.cuda.synchronize()
    hrpp.get_error(bvh)
    assert_same_result(query, got.cpu().numpy(), want)
    gs = hrpp.stats_dict(st)
    for k in ("rays", "invalid", "hits", "traversals"):
        assert gs[k] == ws[k], (k, gs[k], ws[k])
    return gs, ws


def test_wide_tiny_and_edges(hrpp):
    tris, rays = sg.tiny_workload()
    wide_case(hrpp, "tiny", tris, rays)
    rc = rays.copy()
    rc[:, 7] = np.inf
    wide_case(hrpp, "tiny", tris, rc, "closest")
    for lm in (1, 8):
        wide_case(hrpp, f"tiny leaf_max {lm}", tris, rc, "closest", leaf_max=lm)
    # one triangle (the root is a leaf), invalid rays
    one = sg.triangle_soup(3, 1)
    bad = rays[:64].copy()
    bad[::4, 4:7] = 0.0
    bad[1::4, 0] = np.nan
    bad[2::4, 3] = 2.0
    wide_case(hrpp, "one triangle, invalid rays", one, bad)
    wide_case(hrpp, "one triangle, invalid rays", one, bad, "closest")
    import torch
    bvh = hrpp.BVH(tris)
    st = hrpp.new_stats()
    empty = torch.empty((0, 8), dtype=torch.float32, device="cuda")
    hrpp.trace_wide_anyhit(bvh, empty, stats=st)
    hrpp.trace_wide_closest(bvh, empty, stats=st)
    torch.cuda.synchronize()
    assert all(v == 0 for v in hrpp.stats_dict(st).values())


def test_wide_terrain(hrpp, small_terrain):
    tris, prim = small_terrain
    gs, ws = wide_case(hrpp, "terrain primary", tris, prim, "closest")
    assert gs["interior_visited"] < ws["interior_visited"]
    ob = oracle.build_sah(tris)
    he, _ = oracle.trace(ob, tris, prim, query="closest", mode="exact")
    t, p = he[:, 0], he[:, 3].view(np.uint32)
    shadow = sg.shadow_rays_from_hits(tris, prim, t, p, seed=2)
    wide_case(hrpp, "terrain shadow", tris, shadow)
    ao = sg.ao_rays_from_hits(tris, prim[:4000], t[:4000], p[:4000], seed=3, samples=8,
                              tmax=0.05 * sg.scene_diagonal(tris))
    wide_case(hrpp, "terrain ao", tris, ao)


def test_wide_full_size(hrpp, full_terrain):
    w = sg.AT_SCALE
    tris, prim = full_terrain
    wide_case(hrpp, "full primary", tris, prim, "closest", leaf_max=sg.AT_SCALE["leaf_max"],
              passes=sg.AT_SCALE["treelet_passes"])
    ob = oracle.build_sah(tris, leaf_max=sg.AT_SCALE["leaf_max"])
    he, _ = oracle.trace(ob, tris, prim, query="closest", mode="exact")
    shadow = sg.shadow_rays_from_hits(tris, prim, he[:, 0], he[:, 3].view(np.uint32), seed=w["seed"],
                                      light_center=w["light_center"], light_size=w["light_size"])
    wide_case(hrpp, "full shadow", tris, shadow, leaf_max=sg.AT_SCALE["leaf_max"],
              passes=sg.AT_SCALE["treelet_passes"])


# ---------------------------------------------------------------------------
# Replacement policies (FIFO eviction, resident-tag priority)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("policy", [1, 2, 3])
def test_tiny_policies(hrpp, policy):
    tris, rays = sg.tiny_workload()
    for T, W in ((4, 2), (8, 1), (12, 4)):
        _, st = check_case(hrpp, f"tiny policy {policy} T {T} W {W}", tris, rays,
                           pred_cfg=(T, W, 5, 6, 256, 0, 0, 0, policy), calls=2)


@pytest.mark.parametrize("policy", [1, 2, 3])
def test_terrain_policies(hrpp, small_terrain, policy):
    tris, prim = small_terrain
    _, st = check_case(hrpp, f"terrain primary paper policy {policy}", tris, prim, query="closest", mode="paper",
                       pred_cfg=(8, 2, 5, 6, 4096, 0, 0, 0, policy))
    if policy & 1:
        assert st["evictions"] > 0
    if policy & 2:
        assert st["conflicts"] > 0
    check_case(hrpp, f"terrain exact policy {policy}, go-up 1, inline", tris, prim[:30000], query="closest",
               mode="exact", pred_cfg=(6, 3, 4, 4, 2000, 0, 1, 1, policy))
    ob = oracle.build_sah(tris)
    he, _ = oracle.trace(ob, tris, prim, query="closest", mode="exact")
    shadow = sg.shadow_rays_from_hits(tris, prim, he[:, 0], he[:, 3].view(np.uint32), seed=2)
    check_case(hrpp, f"terrain shadow policy {policy}, paper hash", tris, shadow,
               pred_cfg=(7, 4, 5, 5, 4096, 1, 0, 48, policy))


def test_full_size_policy(hrpp, full_terrain):
    w = sg.AT_SCALE
    tris, prim = full_terrain
    pq = w["primary_q"]
    _, st = check_case(hrpp, "full primary paper, FIFO + resident, 2^12 x 4", tris, prim, query="closest",
                       mode="paper", pred_cfg=(12, 4, pq[0], pq[1], pq[2], 0, 0, pq[3], 3, pq[4]),
                       leaf_max=sg.AT_SCALE["leaf_max"], passes=sg.AT_SCALE["treelet_passes"])
    assert st["evictions"] > 0


@pytest.mark.parametrize("inline", [1, 65])
def test_terrain_short_first_epoch(hrpp, small_terrain, inline):
    # one Bayer pass (3,600 of 57,600 primaries) as the first epoch, the rest in
    # one epoch that sees the table the pass left; shadow rays with go-up 1
    tris, prim = small_terrain
    _, st = check_case(hrpp, f"terrain primary paper, first epoch 3600, inline {inline}", tris, prim,
                       query="closest", mode="paper", pred_cfg=(14, 8, 5, 7, 1 << 16, 0, 0, inline, 0, 3600))
    assert st["pred_hits"] > 30000
    check_case(hrpp, f"terrain primary exact, first epoch 1000, inline {inline}", tris, prim[:30000],
               query="closest", mode="exact", pred_cfg=(13, 4, 4, 5, 8192, 0, 0, inline, 0, 1000))
    ob = oracle.build_sah(tris)
    he, _ = oracle.trace(ob, tris, prim, query="closest", mode="exact")
    shadow = sg.shadow_rays_from_hits(tris, prim, he[:, 0], he[:, 3].view(np.uint32), seed=2)
    check_case(hrpp, f"terrain shadow go-up 1, first epoch 7200, inline {inline}", tris, shadow,
               pred_cfg=(14, 8, 6, 3, 1 << 15, 0, 1, inline, 0, 7200))


@pytest.mark.parametrize("inline", [1, 32, 64, 65])
def test_inline_or_queued_fallback_same_results(hrpp, small_terrain, inline):
    # a wave's failing rays traverse at once or through the queue: the
    # schedule must not change results, counters or the table
    tris, prim = small_terrain
    check_case(hrpp, f"terrain primary paper inline {inline}", tris, prim, query="closest", mode="paper",
               pred_cfg=(14, 8, 5, 6, 4096, 0, 0, inline))
    check_case(hrpp, f"terrain primary exact inline {inline}", tris, prim[:30000], query="closest", mode="exact",
               pred_cfg=(13, 4, 4, 5, 3000, 0, 0, inline))
    ob = oracle.build_sah(tris)
    he, _ = oracle.trace(ob, tris, prim, query="closest", mode="exact")
    shadow = sg.shadow_rays_from_hits(tris, prim, he[:, 0], he[:, 3].view(np.uint32), seed=2)
    check_case(hrpp, f"terrain shadow inline {inline} go-up 1", tris, shadow,
               pred_cfg=(14, 8, 5, 6, 4096, 0, 1, inline))


@pytest.mark.parametrize("inline", [1, 32, 65])
def test_small_epochs_one_workgroup(hrpp, small_terrain, inline):
    # epochs of at most 256 rays: the whole call runs in one workgroup, every
    # phase of every epoch (queue included) as the multi-launch form runs it
    tris, prim = small_terrain
    check_case(hrpp, f"terrain primary paper E=256 first 64 inline {inline}", tris, prim[:6000], query="closest",
               mode="paper", pred_cfg=(12, 8, 5, 6, 256, 0, 0, inline, 0, 64), calls=2)
    check_case(hrpp, f"terrain primary exact E=200 inline {inline}", tris, prim[:3000], query="closest",
               mode="exact", pred_cfg=(12, 4, 4, 5, 200, 0, 0, inline))
    ob = oracle.build_sah(tris)
    he, _ = oracle.trace(ob, tris, prim[:5000], query="closest", mode="exact")
    shadow = sg.shadow_rays_from_hits(tris, prim[:5000], he[:, 0], he[:, 3].view(np.uint32), seed=2)
    check_case(hrpp, f"terrain shadow E=128 first 100 go-up 1 fifo inline {inline}", tris, shadow,
               pred_cfg=(12, 8, 6, 3, 128, 0, 1, inline, 1, 100), calls=2)


# ---------------------------------------------------------------------------
# The paper's IEEE-754 bit hash (hash mode 1)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("p", [1, 2, 3, 4, 6, 7])
def test_tiny_paper_hash(hrpp, p):
    tris, rays = sg.tiny_workload()
    check_case(hrpp, f"tiny paper hash p={p}", tris, rays, pred_cfg=(12, 4, p, p, 300, 1), calls=2)


def test_terrain_paper_hash(hrpp, small_terrain):
    tris, prim = small_terrain
    _, st = check_case(hrpp, "terrain primary paper hash p=6", tris, prim, query="closest", mode="paper",
                       pred_cfg=(14, 8, 6, 6, 4096, 1))
    assert st["pred_hits"] > 0
    ob = oracle.build_sah(tris)
    he, _ = oracle.trace(ob, tris, prim, query="closest", mode="exact")
    shadow = sg.shadow_rays_from_hits(tris, prim, he[:, 0], he[:, 3].view(np.uint32), seed=2)
    check_case(hrpp, "terrain shadow paper hash p=5", tris, shadow, pred_cfg=(14, 8, 5, 5, 4096, 1))
    check_case(hrpp, "terrain closest exact paper hash p=3", tris, prim[:20000], query="closest",
               mode="exact", pred_cfg=(10, 2, 3, 3, 1000, 1))


# ---------------------------------------------------------------------------
# Go Up Level >= 1: predicted interior nodes, walked as subtrees
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("g", [1, 2, 3, 64])
def test_tiny_go_up(hrpp, g):
    tris, rays = sg.tiny_workload()
    _, st = check_case(hrpp, f"tiny go-up {g}", tris, rays, pred_cfg=(12, 4, 5, 6, 256, 0, g), calls=2)
    assert st["pred_hits"] > 0
    rc = rays.copy()
    rc[:, 7] = np.inf
    for mode in ("paper", "exact"):
        check_case(hrpp, f"tiny closest {mode} go-up {g}", tris, rc, query="closest", mode=mode,
                   pred_cfg=(12, 4, 5, 6, 256, 0, g), calls=2)


@pytest.mark.parametrize("g", [1, 2])
def test_terrain_go_up(hrpp, small_terrain, g):
    tris, prim = small_terrain
    _, st = check_case(hrpp, f"terrain primary paper go-up {g}", tris, prim, query="closest", mode="paper",
                       pred_cfg=(14, 8, 5, 6, 4096, 0, g))
    assert st["pred_hits"] > 1000
    check_case(hrpp, f"terrain primary exact go-up {g}", tris, prim[:20000], query="closest", mode="exact",
               pred_cfg=(12, 2, 4, 4, 1000, 0, g))
    ob = oracle.build_sah(tris)
    he, _ = oracle.trace(ob, tris, prim, query="closest", mode="exact")
    shadow = sg.shadow_rays_from_hits(tris, prim, he[:, 0], he[:, 3].view(np.uint32), seed=2)
    check_case(hrpp, f"terrain shadow go-up {g}", tris, shadow, pred_cfg=(14, 8, 5, 6, 4096, 0, g))
    check_case(hrpp, f"terrain shadow go-up {g}, one way, paper hash", tris, shadow,
               pred_cfg=(6, 1, 5, 5, 777, 1, g))


def test_full_size_go_up(hrpp, full_terrain):
    w = sg.AT_SCALE
    tris, prim = full_terrain
    pq = w["primary_q"]
    check_case(hrpp, "full primary paper go-up 1", tris, prim, query="closest", mode="paper",
               pred_cfg=(w["log2_entries"], w["ways"], pq[0], pq[1], pq[2], 0, 1, pq[3], 0, pq[4]),
               leaf_max=sg.AT_SCALE["leaf_max"], passes=sg.AT_SCALE["treelet_passes"])


def test_import_validates_slots(hrpp, small_terrain):
    tris, prim = small_terrain
    _say("import validation")
    bvh = hrpp.BVH(tris)
    import torch
    r = torch.from_numpy(prim[:20000]).cuda()
    for g in (0, 2):
        p = hrpp.Predictor(bvh, 12, 4, 5, 6, 4096, go_up_level=g)
        hrpp.trace_closest(bvh, p, r, mode="paper")
        raw = p.export_raw()
        q = hrpp.Predictor(bvh, 12, 4, 5, 6, 4096, go_up_level=g)
        q.import_raw(raw)                                   # round trip
        assert np.array_equal(q.export_raw(), raw)
        tags, slots = p.export()
        used = np.nonzero(tags != np.uint64(0xFFFFFFFFFFFFFFFF))[0]
        assert used.size
        e = int(used[0]) * p.entry_bytes
        bad = raw.copy()
        bad[e + 8:e + 12] = np.frombuffer(np.uint32(0x7FFFFFF0).tobytes(), np.uint8)   # slot out of range
        with pytest.raises(RuntimeError):
            q.import_raw(bad)
        bad = raw.copy()
        bad[e + 8 + 4 * 4:e + 12 + 4 * 4] = 0                 # claim word held
        with pytest.raises(RuntimeError):
            q.import_raw(bad)
        assert np.array_equal(q.export_raw(), raw)           # a refused import copies nothing


# ---------------------------------------------------------------------------
# Edge cases
# ---------------------------------------------------------------------------

def test_edge_cases(hrpp):
    import torch
    tris, rays = sg.tiny_workload()
    _say("edge: n = 0")
    bvh = hrpp.BVH(tris)
    pred = hrpp.Predictor(bvh, 12, 4, 5, 6, 256)
    st = hrpp.new_stats()
    empty = torch.empty((0, 8), dtype=torch.float32, device="cuda")
    hrpp.trace_anyhit(bvh, pred, empty, stats=st)
    hrpp.trace_closest(bvh, pred, empty, stats=st)
    torch.cuda.synchronize()
    assert all(v == 0 for v in hrpp.stats_dict(st).values())
    # invalid rays mixed into valid ones
    bad = rays.copy()
    bad[::7, 4:7] = 0.0
    bad[1::11, 0] = np.nan
    bad[2::13, 7] = bad[2::13, 3]
    bad[3::17, 5] = np.inf
    _, s = check_case(hrpp, "edge invalid rays", tris, bad, pred_cfg=(12, 4, 5, 6, 100))
    assert s["invalid"] > 500
    check_case(hrpp, "edge invalid rays closest", tris, bad, query="closest", mode="exact", pred_cfg=(12, 4, 5, 6, 100))
    # one ray; a single-triangle scene (the root is a leaf); leaf_max 1 and 8
    check_case(hrpp, "edge one ray", tris, rays[:1], pred_cfg=(12, 4, 5, 6, 256))
    one = tris[:1]
    r1 = sg.pack_rays(np.tile(one[0].mean(0) + [0, 0.5, 0], (64, 1)).astype(np.float32),
                      np.tile(np.float32([0.001, -1, 0.002]), (64, 1)), 0.0, np.inf)
    check_case(hrpp, "edge root leaf", one, r1, pred_cfg=(4, 1, 3, 3, 8))
    check_case(hrpp, "edge root leaf closest", one, r1, query="closest", pred_cfg=(4, 1, 3, 3, 8))
    check_case(hrpp, "edge leaf_max 1", tris, rays, pred_cfg=(12, 4, 5, 6, 256), leaf_max=1)
    check_case(hrpp, "edge leaf_max 8", tris, rays, query="closest", mode="paper", pred_cfg=(12, 8, 5, 6, 256),
               leaf_max=8)


def _adversarial_rays(tris, n, seed):
    """Valid rays built to stress the binary32 assumptions both sides share:
    direction components of +-0, subnormal, tiny and huge magnitude (1/d of
    +-inf, huge or subnormal), origins on BVH box planes and on triangle
    planes (slab terms of 0 * inf), tmin of -0 and tmax of +inf."""
    g = np.random.default_rng(seed)
    v = tris.reshape(-1, 3)
    lo, hi = v.min(0), v.max(0)
    specials = np.float32([0.0, -0.0, 1e-45, -1e-45, 1e-39, -1e-39, 1.2e-38, -1.2e-38, 1e-30, -1e30, 3e38])
    tgt = tris[g.integers(0, tris.shape[0], n)].mean(1)
    o = (lo + (hi - lo) * g.uniform(-0.2, 1.2, (n, 3))).astype(np.float32)
    k = g.integers(0, 3, n)
    on_box = g.random(n) < 0.3
    o[on_box, k[on_box]] = np.where(g.random(int(on_box.sum())) < 0.5, lo[k[on_box]], hi[k[on_box]])
    on_tri = g.random(n) < 0.15                       # origin on a vertex's plane
    o[on_tri, k[on_tri]] = v[g.integers(0, v.shape[0], int(on_tri.sum())), k[on_tri]]
    d = (tgt - o).astype(np.float32)
    for axis in range(3):                             # replace components by special values
        m = g.random(n) < 0.3
        d[m, axis] = specials[g.integers(0, specials.size, int(m.sum()))]
    zero = ~np.any(d != 0, axis=1)                    # keep every ray valid
    d[zero, 1] = -1.0
    tmin = np.where(g.random(n) < 0.5, np.float32(-0.0), np.float32(0.0))
    tmax = np.where(g.random(n) < 0.5, np.float32(np.inf), np.float32(1e30))
    r = sg.pack_rays(o, d, 0.0, 0.0)
    r[:, 3], r[:, 7] = tmin, tmax
    return r


def test_adversarial_binary32_rays(hrpp):
    # the GPU's reciprocal, min/max with NaN operands and subnormal handling
    # match the oracle's host arithmetic on rays built to hit those cases
    tris, _ = sg.tiny_workload()
    rays = _adversarial_rays(tris, 4096, 77)
    occ, st = check_case(hrpp, "adversarial binary32, plain any", tris, rays)
    assert st["invalid"] == 0 and 0 < st["hits"] < rays.shape[0]
    check_case(hrpp, "adversarial binary32, hrpp any", tris, rays, pred_cfg=(10, 4, 4, 4, 512), calls=2)
    check_case(hrpp, "adversarial binary32, closest exact", tris, rays, query="closest", mode="exact")
    check_case(hrpp, "adversarial binary32, closest paper", tris, rays, query="closest", mode="paper",
               pred_cfg=(10, 8, 4, 4, 1024, 0, 1))
    terr, _ = sg.terrain_workload(total=30000, width=64, height=36)
    check_case(hrpp, "adversarial binary32, terrain closest exact", terr, _adversarial_rays(terr, 4096, 78),
               query="closest", mode="exact")


def test_determinism_and_reset(hrpp, small_terrain):
    import torch
    tris, prim = small_terrain
    _say("determinism")
    bvh = hrpp.BVH(tris)
    pred = hrpp.Predictor(bvh, 14, 8, 5, 6, 4096)
    r = torch.from_numpy(prim).cuda()
    outs = []
    for _ in range(3):
        pred.reset()
        st = hrpp.new_stats()
        h = hrpp.trace_closest(bvh, pred, r, mode="paper", stats=st)
        torch.cuda.synchronize()
        outs.append((h.cpu().numpy().tobytes(), pred.export_raw().tobytes(), tuple(hrpp.stats_dict(st).items())))
    assert outs[0] == outs[1] == outs[2]
    # export / import round trip restores the trajectory
    pred.reset()
    hrpp.trace_closest(bvh, pred, r[:10000], mode="paper")
    saved = pred.export_raw()
    h1 = hrpp.trace_closest(bvh, pred, r[10000:], mode="paper").cpu().numpy()
    pred.reset()
    pred.import_raw(saved)
    h2 = hrpp.trace_closest(bvh, pred, r[10000:], mode="paper").cpu().numpy()
    assert np.array_equal(h1.view(np.uint32), h2.view(np.uint32))


def test_reset_clears_written_entries(hrpp, small_terrain):
    """A reset empties every entry written since the previous one: the update
    marks the group of each entry it tags while empty and the reset clears the
    marked groups; after an import it clears the whole table.  Tables of few
    and of many used entries, and one smaller than a group."""
    import torch
    tris, prim = small_terrain
    bvh = hrpp.BVH(tris)
    r = torch.from_numpy(prim).cuda()
    empty_tag = np.uint64(0xFFFFFFFFFFFFFFFF)
    for T, W, qo, qd in ((10, 8, 3, 3), (8, 8, 5, 6), (3, 4, 5, 6), (12, 4, 5, 6)):
        _say(f"reset, T {T} W {W} q_o {qo} q_d {qd}")
        pred = hrpp.Predictor(bvh, T, W, qo, qd, 4096)
        fresh = hrpp.Predictor(bvh, T, W, qo, qd, 4096)
        for _ in range(3):
            # two calls between resets: marks persist across calls
            hrpp.trace_closest(bvh, pred, r[:20000], mode="paper")
            hrpp.trace_closest(bvh, pred, r[20000:], mode="paper")
            tags, _ = pred.export()
            assert int((tags != empty_tag).sum()) > 0
            pred.reset()
            assert (pred.export_raw() == 0xFF).all()
        # after the resets the predictor behaves as a new one
        h1 = hrpp.trace_closest(bvh, pred, r, mode="paper").cpu().numpy()
        h2 = hrpp.trace_closest(bvh, fresh, r, mode="paper").cpu().numpy()
        assert np.array_equal(h1.view(np.uint32), h2.view(np.uint32))
        raw = pred.export_raw()
        assert np.array_equal(raw, fresh.export_raw())
        # imported entries carry no marks: the next reset clears everything
        pred.reset()
        pred.import_raw(raw)
        hrpp.trace_closest(bvh, pred, r[:1000], mode="paper")
        pred.reset()
        assert (pred.export_raw() == 0xFF).all()
        pred.close()
        fresh.close()


# ---------------------------------------------------------------------------
# Full size: the 1M-triangle scene at 1920x1080, in the benchmark's launch
# configuration (hit-all predictor 2^20 x 8 for primaries, hit-any predictor
# for shadow rays, a short first epoch then the rest of the frame) and at the
# untuned epochs of 2^17 rays
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def full_terrain():
    return sg.terrain_workload()


@pytest.mark.parametrize("tuned", [True, False])
def test_full_size_primary_and_shadow(hrpp, full_terrain, tuned):
    # the benchmark's launch configuration (autotuned quantisation and epochs),
    # and the untuned reference (q_o 5, q_d 6, epochs of 2^17)
    w = sg.AT_SCALE
    tris, prim = full_terrain
    pq, sq = (w["primary_q"], w["shadow_q"]) if tuned else ((5, 6, 1 << 17, 0, 0), (5, 6, 1 << 17, 0, 0))
    cfg_all = (w["log2_entries"], w["ways"], pq[0], pq[1], pq[2], 0, 0, pq[3], 0, pq[4])
    cfg_any = (w["log2_entries"], w["ways"], sq[0], sq[1], sq[2], 0, 0, sq[3], 0, sq[4])
    _, st = check_case(hrpp, "full primary paper", tris, prim, query="closest", mode="paper", pred_cfg=cfg_all,
                       leaf_max=sg.AT_SCALE["leaf_max"], passes=sg.AT_SCALE["treelet_passes"])
    assert st["rays"] == 1920 * 1080
    ob = oracle.build_sah(tris, leaf_max=sg.AT_SCALE["leaf_max"])
    he, _ = oracle.trace(ob, tris, prim, query="closest", mode="exact")
    check_case(hrpp, "full primary exact (plain)", tris, prim, query="closest", mode="exact",
               leaf_max=sg.AT_SCALE["leaf_max"], passes=sg.AT_SCALE["treelet_passes"])
    shadow = sg.shadow_rays_from_hits(tris, prim, he[:, 0], he[:, 3].view(np.uint32), seed=w["seed"],
                                      light_center=w["light_center"], light_size=w["light_size"])
    check_case(hrpp, "full shadow plain", tris, shadow, leaf_max=sg.AT_SCALE["leaf_max"],
               passes=sg.AT_SCALE["treelet_passes"])
    check_case(hrpp, "full shadow hrpp", tris, shadow, pred_cfg=cfg_any, leaf_max=sg.AT_SCALE["leaf_max"],
               passes=sg.AT_SCALE["treelet_passes"])


def test_full_size_progressive_frames(hrpp, full_terrain):
    # the benchmark's warm-table measurement: successive frames of jittered
    # row-major primaries (and their shadow rays) traced with the tables kept,
    # one epoch per frame; every frame against the oracle, which carries its
    # own tables across the frames in the same way
    import torch
    w = sg.AT_SCALE
    tris, _ = full_terrain
    bvh = hrpp.BVH(tris, leaf_max=sg.AT_SCALE["leaf_max"], treelet_passes=sg.AT_SCALE["treelet_passes"])
    ob = oracle.build_sah(tris, leaf_max=sg.AT_SCALE["leaf_max"], treelet_passes=sg.AT_SCALE["treelet_passes"])
    vtx = oracle.bvh_vertices(tris, ob)
    pq, sq = w["primary_q"], w["shadow_q"]
    E = 1 << 21
    pa = hrpp.Predictor(bvh, log2_entries=w["log2_entries"], ways=w["ways"], origin_bits=pq[0], dir_bits=pq[1],
                        epoch_rays=E, inline_lanes=1)
    pb = hrpp.Predictor(bvh, log2_entries=w["log2_entries"], ways=w["ways"], origin_bits=sq[0], dir_bits=sq[1],
                        epoch_rays=E, inline_lanes=1)
    ta = oracle.Table(w["log2_entries"], w["ways"], pq[0], pq[1])
    tb = oracle.Table(w["log2_entries"], w["ways"], sq[0], sq[1])
    cam = sg.camera_for(w["width"], w["height"])
    for k, off in enumerate(sg.PROGRESSIVE_OFFSETS[:2]):
        _say(f"progressive frame {k}, offset {off}")
        prim, _ = cam.rays("rowmajor", off)
        got, gs = gpu_run(hrpp, bvh, prim, "closest", "paper", pa)
        want, ws = oracle.trace(ob, tris, prim, query="closest", mode="paper", table=ta, epoch=E, vtx=vtx)
        assert_same_result("closest", got, want)
        assert {k2: gs[k2] for k2 in ws} == ws
        assert_same_table(pa, ta)
        if k > 0:
            assert ws["pred_hits"] > 0.9 * prim.shape[0]      # the previous frame's entries predict
        he, _ = oracle.trace(ob, tris, prim, query="closest", mode="exact", vtx=vtx)
        shadow = sg.shadow_rays_from_hits(tris, prim, he[:, 0], he[:, 3].view(np.uint32), seed=w["seed"] + 1 + k,
                                          light_center=w["light_center"], light_size=w["light_size"])
        got, gs = gpu_run(hrpp, bvh, shadow, "any", "paper", pb)
        want, ws = oracle.trace(ob, tris, shadow, query="any", table=tb, epoch=E, vtx=vtx)
        assert_same_result("any", got, want)
        assert {k2: gs[k2] for k2 in ws} == ws
        assert_same_table(pb, tb)
    torch.cuda.synchronize()


@pytest.mark.parametrize("cfg", [
    (sg.INCOHERENT["log2_entries"], sg.INCOHERENT["ways"], sg.INCOHERENT["origin_bits"], sg.INCOHERENT["dir_bits"],
     sg.INCOHERENT["epoch"], 0, 0, sg.INCOHERENT["inline_lanes"], 0,
     sg.INCOHERENT["first_epoch"]),                                   # the benchmark's AO predictor
    (16, 8, 3, 3, 1 << 17, 1),     # sweep corners, the IEEE-754 bit hash
    (22, 8, 7, 7, 1 << 17, 1),
])
def test_full_size_ao(hrpp, full_terrain, cfg):
    # the incoherent workload: 1280x720 primaries x 8 AO rays (7,372,800)
    wi = sg.INCOHERENT
    tris, _ = full_terrain
    cam, _ = sg.camera_for(wi["width"], wi["height"]).rays("rowmajor")
    ob = oracle.build_sah(tris, leaf_max=sg.AT_SCALE["leaf_max"])
    hh, _ = oracle.trace(ob, tris, cam, query="closest", mode="exact")
    ao = sg.ao_rays_from_hits(tris, cam, hh[:, 0], hh[:, 3].view(np.uint32), seed=wi["seed"],
                              samples=wi["samples"], tmax=wi["tmax_frac"] * sg.scene_diagonal(tris))
    assert ao.shape[0] == 7372800
    _, st = check_case(hrpp, f"full AO {cfg}", tris, ao, pred_cfg=cfg, leaf_max=sg.AT_SCALE["leaf_max"],
                       passes=sg.AT_SCALE["treelet_passes"])
    assert st["rays"] == 7372800


def test_maximum_epoch_and_large_table(hrpp, full_terrain):
    # the largest epoch (2^22 rays) over the 7,372,800 AO rays (one full epoch
    # and a ragged one) with a 2^24-entry table, queue-only and in-place fallback
    wi = sg.INCOHERENT
    tris, _ = full_terrain
    cam, _ = sg.camera_for(wi["width"], wi["height"]).rays("rowmajor")
    ob = oracle.build_sah(tris, leaf_max=sg.AT_SCALE["leaf_max"])
    hh, _ = oracle.trace(ob, tris, cam, query="closest", mode="exact")
    ao = sg.ao_rays_from_hits(tris, cam, hh[:, 0], hh[:, 3].view(np.uint32), seed=wi["seed"],
                              samples=wi["samples"], tmax=wi["tmax_frac"] * sg.scene_diagonal(tris))
    for inline in (65, 1):
        _, st = check_case(hrpp, f"AO, epoch 2^22, table 2^24 x 4, inline {inline}", tris, ao,
                           pred_cfg=(24, 4, 5, 6, 1 << 22, 0, 0, inline), leaf_max=sg.AT_SCALE["leaf_max"],
                           passes=sg.AT_SCALE["treelet_passes"])
        assert st["rays"] == 7372800 and st["pred_hits"] > 0


def test_random_configurations(hrpp):
    # random predictor configurations on small random scenes, every one against
    # the oracle: hash mode, go-up level, replacement policy, fallback split,
    # epoch (ragged) and first epoch, table shape, query and closest-hit mode
    g = np.random.default_rng(2024)
    gf = np.random.default_rng(2025)          # first epochs (drawn apart, so the other draws stay as they were)
    for case in range(40):
        seed = int(g.integers(1, 1 << 30))
        n_tris = int(g.integers(1, 3000))
        tris = sg.mixed_scene(seed, n_tris) if n_tris > 50 else sg.triangle_soup(seed, n_tris)
        sh, ao = sg.secondary_rays_on_surface(tris, int(g.integers(1, 6000)), seed + 1)
        rays = np.concatenate([sh, ao])
        query = ["any", "closest"][int(g.integers(0, 2))]
        mode = ["paper", "exact"][int(g.integers(0, 2))]
        if query == "closest" and g.random() < 0.5:
            rays = rays.copy()
            rays[:, 7] = np.inf
        hm = int(g.integers(0, 2))
        q = int(g.integers(1, 8)) if hm else None
        qo, qd = (q, q) if hm else (int(g.integers(1, 9)), int(g.integers(1, 9)))
        cfg = (int(g.integers(1, 15)), int(g.integers(1, 9)), qo, qd, int(g.integers(1, 3000)), hm,
               int(g.choice([0, 0, 1, 2, 5])), int(g.choice([0, 1, 16, 48, 64, 65])), int(g.integers(0, 4)))
        cfg = cfg + ((0 if gf.random() < 0.4 else int(gf.integers(1, cfg[4] + 1))),)
        check_case(hrpp, f"random {case}", tris, rays, query=query, mode=mode, pred_cfg=cfg,
                   calls=int(g.integers(1, 3)), leaf_max=int(g.choice([1, 2, 4, 8])))


def test_epoch_aligned_split_calls_equal_one_call(hrpp, small_terrain):
    # ray ids are call-relative and each call starts an epoch, so tracing the
    # rays in two calls split at an epoch boundary computes exactly what one
    # call computes (results, the method's counters, the table)
    import torch
    tris, prim = small_terrain
    _say("split calls")
    bvh = hrpp.BVH(tris)
    r = torch.from_numpy(prim).cuda()
    E = 4096
    for query, mode in (("closest", "paper"), ("any", "paper"), ("closest", "exact")):
        outs = []
        for split in (None, 3 * E):
            pred = hrpp.Predictor(bvh, 14, 8, 5, 6, E, inline_lanes=16)
            st = hrpp.new_stats()
            parts = [(0, r.shape[0])] if split is None else [(0, split), (split, r.shape[0])]
            if query == "any":
                out = torch.empty(r.shape[0], dtype=torch.uint8, device="cuda")
                for a, b in parts:
                    hrpp.trace_anyhit(bvh, pred, r[a:b], out=out[a:b], stats=st)
            else:
                out = torch.empty((r.shape[0], 4), dtype=torch.float32, device="cuda")
                for a, b in parts:
                    hrpp.trace_closest(bvh, pred, r[a:b], mode=mode, out=out[a:b], stats=st)
            torch.cuda.synchronize()
            d = {k: v for k, v in hrpp.stats_dict(st).items() if k not in hrpp.SCHEDULE_STATS}
            outs.append((out.cpu().numpy().tobytes(), pred.export_raw().tobytes(), d))
        assert outs[0] == outs[1], query


def test_results_do_not_depend_on_stats(hrpp, small_terrain):
    # the benchmark times the path without counters; it must compute the same
    import torch
    tris, prim = small_terrain
    _say("stats on/off")
    bvh = hrpp.BVH(tris)
    r = torch.from_numpy(prim).cuda()
    res = []
    for with_stats in (True, False):
        pa = hrpp.Predictor(bvh, 14, 8, 5, 6, 4096)
        st = hrpp.new_stats() if with_stats else None
        h = hrpp.trace_closest(bvh, pa, r, mode="paper", stats=st).cpu().numpy()
        o = hrpp.trace_anyhit(bvh, pa, r, stats=st).cpu().numpy()
        hp = hrpp.trace_closest(bvh, None, r, mode="exact", stats=st).cpu().numpy()
        res.append((h.tobytes(), o.tobytes(), hp.tobytes(), pa.export_raw().tobytes()))
    assert res[0] == res[1]
