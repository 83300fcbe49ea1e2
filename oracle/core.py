"""ctypes wrapper of the C oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hrpp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

STAT_NAMES = [
    "rays", "invalid", "hits", "lookups", "positives", "pred_hits", "false_pos", "traversals",
    "nodes_visited", "interior_visited", "leaf_visited", "box_tests", "tri_tests", "nodes_skipped",
    "records", "tag_claims", "leaf_inserts", "dropped", "conflicts", "pred_leaf_visited", "pred_tri_tests",
    "pred_box_tests", "evictions",
]
STATS_SLOTS = 24
NONE32 = 0xFFFFFFFF


def lib_path() -> str:
    return _LIB


def build_library(force: bool = True) -> str:
    """Compile the oracle (gcc, binary32 without contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-shared", "-fPIC", "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _L():
    global _lib
    if _lib is None:
        alt = os.environ.get("HRPP_ORACLE_LIB")   # another build of the same source (a sanitizer build)
        if alt:
            _lib = C.CDLL(alt)
            return _lib
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build_library(force=True)
        _lib = C.CDLL(_LIB)
    return _lib


class _OrcBVH(C.Structure):
    _fields_ = [("num_nodes", C.c_uint32), ("num_tris", C.c_uint32),
                ("box", C.c_void_p), ("right", C.c_void_p), ("first", C.c_void_p),
                ("count", C.c_void_p), ("depth", C.c_void_p), ("perm", C.c_void_p)]


def _p(a: np.ndarray):
    return C.c_void_p(a.ctypes.data) if a is not None else None


@dataclass
class CanonBVH:
    """Canonical depth-first pre-order BVH (left child = next node)."""
    box: np.ndarray      # [m, 6] float32
    right: np.ndarray    # [m] uint32 (0xFFFFFFFF for leaves)
    first: np.ndarray    # [m] uint32
    count: np.ndarray    # [m] uint32
    depth: np.ndarray    # [m] uint32
    perm: np.ndarray     # [n] uint32  BVH position -> original primitive id

    @property
    def num_nodes(self) -> int:
        return int(self.box.shape[0])

    @property
    def num_tris(self) -> int:
        return int(self.perm.shape[0])

    def is_leaf(self) -> np.ndarray:
        return self.right == NONE32

    def leaf_ids(self) -> np.ndarray:
        lf = self.is_leaf()
        return (self.first[lf].astype(np.uint64) << 3 | (self.count[lf].astype(np.uint64) - 1)).astype(np.uint32)

    def max_depth(self) -> int:
        return int(self.depth[self.is_leaf()].max())

    def _struct(self):
        s = _OrcBVH(self.num_nodes, self.num_tris, self.box.ctypes.data, self.right.ctypes.data,
                    self.first.ctypes.data, self.count.ctypes.data, self.depth.ctypes.data,
                    self.perm.ctypes.data)
        return s


def _empty_bvh(n: int):
    m = 2 * n - 1
    return _OrcBVH(0, n, None, None, None, None, None, None), dict(
        box=np.zeros((m, 6), np.float32), right=np.zeros(m, np.uint32), first=np.zeros(m, np.uint32),
        count=np.zeros(m, np.uint32), depth=np.zeros(m, np.uint32), perm=np.zeros(n, np.uint32))


def _run_build(fn, tris, *args) -> CanonBVH:
    tris = np.ascontiguousarray(tris, np.float32).reshape(-1, 9)
    n = tris.shape[0]
    s, arrs = _empty_bvh(n)
    for k in ("box", "right", "first", "count", "depth", "perm"):
        setattr(s, k, arrs[k].ctypes.data)
    rc = fn(_p(tris), C.c_uint32(n), *[C.c_uint32(a) for a in args], C.byref(s))
    if rc != 0:
        raise ValueError(f"oracle BVH build failed ({rc})")
    m = s.num_nodes
    return CanonBVH(arrs["box"][:m].copy(), arrs["right"][:m].copy(), arrs["first"][:m].copy(),
                    arrs["count"][:m].copy(), arrs["depth"][:m].copy(), arrs["perm"].copy())


def build_sah(tris: np.ndarray, leaf_max: int = 4, bins: int = 32, max_depth: int = 64,
              treelet_passes: int = 0) -> CanonBVH:
    """Deterministic binned-SAH BVH (the reading both sides implement); with
    treelet_passes >= 1, that many passes of treelet restructuring after it."""
    if treelet_passes:
        return _run_build(_L().orc_build_sah_treelet, tris, leaf_max, bins, max_depth, treelet_passes)
    return _run_build(_L().orc_build_sah, tris, leaf_max, bins, max_depth)


def build_median(tris: np.ndarray, leaf_max: int = 4, max_depth: int = 100) -> CanonBVH:
    """A differently shaped BVH (median splits) for shape-independence pins."""
    return _run_build(_L().orc_build_median, tris, leaf_max, max_depth)


def build_lbvh(tris: np.ndarray, leaf_max: int = 4, max_depth: int = 64, treelet_passes: int = 0) -> CanonBVH:
    """Linear BVH: Morton order of the triangle centres, radix-tree splits;
    with treelet_passes >= 1, that many passes of treelet restructuring."""
    if treelet_passes:
        return _run_build(_L().orc_build_lbvh_treelet, tris, leaf_max, max_depth, treelet_passes)
    return _run_build(_L().orc_build_lbvh, tris, leaf_max, max_depth)


def lbvh_codes(tris: np.ndarray) -> np.ndarray:
    """The 63-bit Morton code of every triangle (original order)."""
    tris = np.ascontiguousarray(tris, np.float32).reshape(-1, 9)
    out = np.zeros(tris.shape[0], np.uint64)
    _L().orc_lbvh_codes(_p(tris), C.c_uint32(tris.shape[0]), _p(out))
    return out


def bvh_vertices(tris: np.ndarray, bvh: CanonBVH) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(tris, np.float32).reshape(-1, 9)[bvh.perm])


class Table:
    """Predictor table: ``tags[N]`` (uint64, all-ones = empty) and ``slots[N, W]``.

    ``hash_mode`` 0: grid origin + octahedral direction (qo, qd bits);
    1: the paper's IEEE-754 bit hash with precision qo in 1..7 (qd must equal qo).
    ``go_up`` 0: slots hold leaf ids; g >= 1: canonical node indices of the
    node g levels above the result leaf (the root if the leaf is shallower).
    ``policy`` bit 0: FIFO eviction within an entry; bit 1: an entry's
    resident tag keeps the entry (0 = the paper's: no eviction).
    """

    def __init__(self, log2n: int, ways: int, qo: int, qd: int, hash_mode: int = 0, go_up: int = 0,
                 policy: int = 0):
        self.log2n, self.W, self.qo, self.qd, self.hash_mode = log2n, ways, qo, qd, hash_mode
        self.go_up, self.policy = go_up, policy
        self.tags = np.full(1 << log2n, np.uint64(0xFFFFFFFFFFFFFFFF), np.uint64)
        self.slots = np.full((1 << log2n, ways), NONE32, np.uint32)

    def reset(self):
        self.tags[:] = np.uint64(0xFFFFFFFFFFFFFFFF)
        self.slots[:] = NONE32

    def copy(self) -> "Table":
        t = Table(self.log2n, self.W, self.qo, self.qd, self.hash_mode, self.go_up, self.policy)
        t.tags[:] = self.tags
        t.slots[:] = self.slots
        return t


def stats_dict(arr: np.ndarray) -> dict:
    return {k: int(arr[i]) for i, k in enumerate(STAT_NAMES)}


def trace(bvh: CanonBVH, tris: np.ndarray, rays: np.ndarray, query: str = "any", mode: str = "paper",
          table: Table | None = None, epoch: int = 1 << 17, nthreads: int = 0, vtx: np.ndarray | None = None,
          outcome: np.ndarray | None = None, first_epoch: int = 0):
    """Run the oracle.  Returns ``(result, stats)``.

    Epochs of ``epoch`` rays in ray order, the first of them ``first_epoch``
    rays long (0: ``epoch``; at most ``epoch``).

    ``result`` is a uint8 occlusion array (any-hit) or a ``[n, 4]`` float32
    array (t, u, v, prim bits) for closest hit.  ``table`` is updated in place.
    ``outcome`` (uint8 [n], optional) receives 0 invalid, 1 traversed without a
    positive prediction, 2 prediction hit, 3 false positive.
    """
    rays = np.ascontiguousarray(rays, np.float32).reshape(-1, 8)
    n = rays.shape[0]
    if vtx is None:
        vtx = bvh_vertices(tris, bvh)
    closest = query == "closest"
    occ = None if closest else np.zeros(n, np.uint8)
    hits = np.zeros((n, 4), np.float32) if closest else None
    stats = np.zeros(STATS_SLOTS, np.uint64)
    s = bvh._struct()
    if table is not None:
        tg, sl, l2, W, qo, qd = table.tags, table.slots, table.log2n, table.W, table.qo, table.qd
        hm, gu, pol = table.hash_mode, table.go_up, table.policy
    else:
        tg = sl = None
        l2 = W = qo = qd = hm = gu = pol = 0
    rc = _L().orc_trace(C.byref(s), _p(vtx), _p(rays), C.c_uint32(n), C.c_int(1 if closest else 0),
                        C.c_int(1 if mode == "exact" else 0), _p(tg), _p(sl), C.c_uint32(l2), C.c_uint32(W),
                        C.c_uint32(qo), C.c_uint32(qd), C.c_uint32(epoch), _p(occ), _p(hits), _p(stats),
                        _p(outcome), C.c_int(nthreads), C.c_uint32(hm), C.c_uint32(gu),
                        C.c_uint32(pol), C.c_uint32(first_epoch))
    if rc != 0:
        raise ValueError("oracle trace rejected its arguments")
    return (hits if closest else occ), stats_dict(stats)


def brute_force(tris: np.ndarray, rays: np.ndarray, closest: bool = False, nthreads: int = 0):
    """All-triangle binary32 test: any-hit flags, or exact closest (t,u,v,prim bits)."""
    tris = np.ascontiguousarray(tris, np.float32).reshape(-1, 9)
    rays = np.ascontiguousarray(rays, np.float32).reshape(-1, 8)
    n = rays.shape[0]
    occ = np.zeros(n, np.uint8)
    hits = np.zeros((n, 4), np.float32)
    _L().orc_brute_force(_p(tris), C.c_uint32(tris.shape[0]), _p(rays), C.c_uint32(n), C.c_int(int(closest)),
                         _p(occ), _p(hits), C.c_int(nthreads))
    return hits if closest else occ


def hash_rays(root_box: np.ndarray, qo: int, qd: int, log2n: int, rays: np.ndarray, hash_mode: int = 0):
    rays = np.ascontiguousarray(rays, np.float32).reshape(-1, 8)
    box = np.ascontiguousarray(root_box, np.float32).reshape(6)
    n = rays.shape[0]
    keys = np.zeros(n, np.uint64)
    idx = np.zeros(n, np.uint32)
    _L().orc_hash(_p(box), C.c_uint32(qo), C.c_uint32(qd), C.c_uint32(log2n), _p(rays), C.c_uint32(n),
                  _p(keys), _p(idx), C.c_uint32(hash_mode))
    return keys, idx


def mt(tri: np.ndarray, ray: np.ndarray):
    """Single binary32 Moller-Trumbore test: returns (hit, t, u, v)."""
    tri = np.ascontiguousarray(tri, np.float32).reshape(9)
    ray = np.ascontiguousarray(ray, np.float32).reshape(8)
    out = np.zeros(3, np.float32)
    h = _L().orc_mt(_p(tri), _p(ray), _p(out))
    return bool(h), float(out[0]), float(out[1]), float(out[2])


def slab(box: np.ndarray, ray: np.ndarray, tcur: float):
    """Single slab test of a box against [ray.tmin, tcur]: returns (hit, tnear)."""
    box = np.ascontiguousarray(box, np.float32).reshape(6)
    ray = np.ascontiguousarray(ray, np.float32).reshape(8)
    tn = C.c_float(0.0)
    fn = _L().orc_slab
    fn.argtypes = [C.c_void_p, C.c_void_p, C.c_float, C.POINTER(C.c_float)]
    h = fn(_p(box), _p(ray), C.c_float(tcur), C.byref(tn))
    return bool(h), float(tn.value)
