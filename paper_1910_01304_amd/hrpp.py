"""Thin ctypes binding of libhrpp.so (include/hrpp.h).

Argument marshalling only: every step of the query path runs in the
library's HIP kernels.  PyTorch provides device memory (``torch.empty`` on
``cuda``) and the current stream.  The binding refuses to run without the
compiled library -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhrpp.so")

STAT_NAMES = [
    "rays", "invalid", "hits", "lookups", "positives", "pred_hits", "false_pos", "traversals",
    "nodes_visited", "interior_visited", "leaf_visited", "box_tests", "tri_tests", "nodes_skipped",
    "records", "tag_claims", "leaf_inserts", "dropped", "conflicts", "pred_leaf_visited", "pred_tri_tests",
    "pred_box_tests", "evictions",
    # schedule counters (how much fallback work ran in the queue kernel), not part of the method
    "queue_traversals", "queue_interior_visited", "queue_tri_tests", "queue_records", "empty_lookups",
    "empty_rays", "empty_interior_visited", "empty_tri_tests", "empty_records",
]
SCHEDULE_STATS = ("queue_traversals", "queue_interior_visited", "queue_tri_tests", "queue_records",
                  "empty_lookups", "empty_rays", "empty_interior_visited", "empty_tri_tests", "empty_records")
STATS_SLOTS = 32
CLOSEST_MODES = {"paper": 0, "exact": 1}
EXPORTED = [
    "hrpp_bvh_required_bytes", "hrpp_build_bvh", "hrpp_bvh_build_host", "hrpp_bvh_device_bytes",
    "hrpp_bvh_upload", "hrpp_bvh_info", "hrpp_bvh_export", "hrpp_bvh_destroy",
    "hrpp_predictor_required_bytes", "hrpp_predictor_table_bytes", "hrpp_predictor_create",
    "hrpp_predictor_reset", "hrpp_predictor_export", "hrpp_predictor_import", "hrpp_predictor_destroy",
    "hrpp_trace_anyhit", "hrpp_trace_closest", "hrpp_get_error", "hrpp_status_string",
    "hrpp_profile_start", "hrpp_profile_stop", "hrpp_batch_required_bytes", "hrpp_batch_create",
    "hrpp_batch_launch", "hrpp_batch_destroy", "hrpp_serve_create", "hrpp_serve_submit", "hrpp_serve_poll",
    "hrpp_serve_wait_all", "hrpp_serve_pool_peak", "hrpp_serve_destroy", "hrpp_bvh_wide_info",
    "hrpp_bvh_wide_export", "hrpp_trace_wide_anyhit", "hrpp_trace_wide_closest",
    "hrpp_bvh_device_build_scratch_bytes", "hrpp_build_bvh_device", "hrpp_serve_add_scene",
    "hrpp_serve_remove_scene", "hrpp_build_bvh_device_static", "hrpp_serve_held",
    "hrpp_profile_touch",
]


class HrppError(RuntimeError):
    pass


class _BvhDesc(C.Structure):
    _fields_ = [("leaf_max", C.c_uint32), ("sah_bins", C.c_uint32), ("max_depth", C.c_uint32),
                ("treelet_passes", C.c_uint32)]


class _PredDesc(C.Structure):
    _fields_ = [("log2_entries", C.c_uint32), ("ways", C.c_uint32), ("origin_bits", C.c_uint32),
                ("dir_bits", C.c_uint32), ("epoch_rays", C.c_uint32), ("hash_mode", C.c_uint32),
                ("go_up_level", C.c_uint32), ("inline_lanes", C.c_uint32), ("replace_policy", C.c_uint32),
                ("first_epoch_rays", C.c_uint32)]


class _KernelTime(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_uint64), ("total_ms", C.c_double)]


class _BatchJob(C.Structure):
    _fields_ = [("bvh", C.c_void_p), ("pred", C.c_void_p), ("rays", C.c_void_p), ("n", C.c_uint32),
                ("query", C.c_uint32), ("mode", C.c_uint32), ("out", C.c_void_p), ("stats", C.c_void_p)]


class _ServeScene(C.Structure):
    _fields_ = [("bvh", C.c_void_p), ("any_preds", C.c_void_p), ("n_any", C.c_uint32),
                ("closest_preds", C.c_void_p), ("n_closest", C.c_uint32)]


class _RequestInfo(C.Structure):
    _fields_ = [("state", C.c_uint32), ("status", C.c_int), ("queue_ms", C.c_double), ("service_ms", C.c_double),
                ("latency_ms", C.c_double)]


class _Canon(C.Structure):
    _fields_ = [("box", C.c_void_p), ("right", C.c_void_p), ("first_tri", C.c_void_p),
                ("count", C.c_void_p), ("depth", C.c_void_p), ("tri_perm", C.c_void_p)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libhrpp.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise HrppError(f"HRPP HIP library not built: {path} is missing (run python -m paper_1910_01304_amd.build)")
    lib = C.CDLL(path)
    vp, u32, sz = C.c_void_p, C.c_uint32, C.c_size_t
    lib.hrpp_bvh_required_bytes.restype = sz
    lib.hrpp_bvh_required_bytes.argtypes = [u32, vp]
    lib.hrpp_build_bvh.argtypes = [vp, u32, vp, vp, sz, vp, C.POINTER(vp)]
    lib.hrpp_bvh_build_host.argtypes = [vp, u32, vp, C.POINTER(vp)]
    lib.hrpp_bvh_device_bytes.restype = sz
    lib.hrpp_bvh_device_bytes.argtypes = [vp]
    lib.hrpp_bvh_upload.argtypes = [vp, vp, sz, vp]
    lib.hrpp_bvh_device_build_scratch_bytes.restype = sz
    lib.hrpp_bvh_device_build_scratch_bytes.argtypes = [u32]
    lib.hrpp_build_bvh_device.argtypes = [vp, u32, vp, vp, sz, vp, sz, vp, C.POINTER(vp)]
    lib.hrpp_build_bvh_device_static.argtypes = [vp, u32, vp, vp, sz, vp, C.POINTER(vp)]
    lib.hrpp_bvh_info.argtypes = [vp, C.POINTER(u32), C.POINTER(u32), C.POINTER(u32)]
    lib.hrpp_bvh_export.argtypes = [vp, vp]
    lib.hrpp_bvh_destroy.argtypes = [vp]
    lib.hrpp_bvh_destroy.restype = None
    lib.hrpp_predictor_required_bytes.restype = sz
    lib.hrpp_predictor_required_bytes.argtypes = [vp]
    lib.hrpp_predictor_table_bytes.restype = sz
    lib.hrpp_predictor_table_bytes.argtypes = [vp]
    lib.hrpp_predictor_create.argtypes = [vp, vp, vp, sz, vp, C.POINTER(vp)]
    lib.hrpp_predictor_reset.argtypes = [vp, vp]
    lib.hrpp_predictor_export.argtypes = [vp, vp, sz, vp]
    lib.hrpp_predictor_import.argtypes = [vp, vp, sz, vp]
    lib.hrpp_predictor_destroy.argtypes = [vp]
    lib.hrpp_predictor_destroy.restype = None
    lib.hrpp_trace_anyhit.argtypes = [vp, vp, vp, u32, vp, vp, vp]
    lib.hrpp_trace_closest.argtypes = [vp, vp, vp, u32, u32, vp, vp, vp]
    lib.hrpp_get_error.argtypes = [vp, vp]
    lib.hrpp_bvh_wide_info.argtypes = [vp, C.POINTER(u32), C.POINTER(u32), C.POINTER(u32), C.POINTER(u32)]
    lib.hrpp_bvh_wide_export.argtypes = [vp, vp, sz]
    lib.hrpp_trace_wide_anyhit.argtypes = [vp, vp, u32, vp, vp, vp]
    lib.hrpp_trace_wide_closest.argtypes = [vp, vp, u32, vp, vp, vp]
    lib.hrpp_profile_stop.argtypes = [vp, u32, C.POINTER(u32)]
    lib.hrpp_profile_touch.argtypes = [vp, vp, vp, sz, vp]
    lib.hrpp_batch_required_bytes.restype = sz
    lib.hrpp_batch_required_bytes.argtypes = [u32]
    lib.hrpp_batch_create.argtypes = [vp, u32, vp, sz, vp, C.POINTER(vp)]
    lib.hrpp_batch_launch.argtypes = [vp, u32, vp]
    lib.hrpp_batch_destroy.argtypes = [vp]
    lib.hrpp_batch_destroy.restype = None
    lib.hrpp_serve_create.argtypes = [vp, u32, u32, vp, sz, C.POINTER(vp)]
    lib.hrpp_serve_submit.argtypes = [vp, u32, u32, vp, u32, vp, C.POINTER(C.c_uint64)]
    lib.hrpp_serve_add_scene.argtypes = [vp, vp, C.POINTER(u32)]
    lib.hrpp_serve_remove_scene.argtypes = [vp, u32]
    lib.hrpp_serve_poll.argtypes = [vp, C.c_uint64, vp]
    lib.hrpp_serve_wait_all.argtypes = [vp]
    lib.hrpp_serve_pool_peak.argtypes = [vp, C.POINTER(sz)]
    lib.hrpp_serve_held.argtypes = [vp, C.POINTER(C.c_uint64)]
    lib.hrpp_serve_destroy.argtypes = [vp]
    lib.hrpp_serve_destroy.restype = None
    lib.hrpp_status_string.restype = C.c_char_p
    lib.hrpp_status_string.argtypes = [C.c_int]
    _lib = lib
    return lib


def _check(status: int, what: str):
    if status != 0:
        msg = load_library().hrpp_status_string(status).decode()
        raise HrppError(f"{what}: {msg} ({status})")


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _aligned(nbytes: int, device):
    """A uint8 device buffer with a 256-byte aligned view of nbytes."""
    raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-raw.data_ptr()) % 256
    return raw, raw[off:off + nbytes]


class BVH:
    """A BVH built on the host and resident in device memory."""

    def __init__(self, tris: np.ndarray, leaf_max: int = 4, sah_bins: int = 32, max_depth: int = 64,
                 device: str | None = "cuda", treelet_passes: int = 0):
        """Build the tree on the host (binned SAH, then `treelet_passes` passes of treelet
        restructuring); upload it to ``device`` unless None."""
        lib = load_library()
        v = np.ascontiguousarray(np.asarray(tris, np.float32).reshape(-1, 9))
        self.num_tris = int(v.shape[0])
        self.desc = _BvhDesc(leaf_max, sah_bins, max_depth, treelet_passes)
        h = C.c_void_p()
        _check(lib.hrpp_bvh_build_host(v.ctypes.data, self.num_tris, C.byref(self.desc), C.byref(h)),
               "hrpp_bvh_build_host")
        self.handle = h
        nn, nt, md = C.c_uint32(), C.c_uint32(), C.c_uint32()
        _check(lib.hrpp_bvh_info(h, C.byref(nn), C.byref(nt), C.byref(md)), "hrpp_bvh_info")
        self.num_nodes, self.max_depth = nn.value, md.value
        self.device_bytes = lib.hrpp_bvh_device_bytes(h)
        self.buffer = None
        if device is not None:
            self.upload(device)

    @classmethod
    def build_on_device(cls, verts: torch.Tensor, leaf_max: int = 4, max_depth: int = 64,
                        static_scratch: bool = False, treelet_passes: int = 0) -> "BVH":
        """Linear BVH built on the GPU from a device tensor of [n, 9] (or [n, 3, 3]) float32 vertices.

        static_scratch: build in the library's static scratch (hrpp_build_bvh_device_static) instead of a
        scratch buffer allocated here.  treelet_passes: passes of treelet restructuring (0 = none)."""
        lib = load_library()
        if not (isinstance(verts, torch.Tensor) and verts.is_cuda and verts.dtype == torch.float32):
            raise HrppError("build_on_device takes a float32 device tensor")
        v = verts.reshape(-1, 9).contiguous()
        self = cls.__new__(cls)
        self.num_tris = int(v.shape[0])
        self.desc = _BvhDesc(leaf_max, 32, max_depth, treelet_passes)
        if static_scratch:
            # the library's static scratch: the build allocates no scratch
            self.device_bytes = lib.hrpp_bvh_required_bytes(self.num_tris, C.byref(self.desc))
            self._raw, self.buffer = _aligned(self.device_bytes, v.device)
            h = C.c_void_p()
            self.handle = None
            _check(lib.hrpp_build_bvh_device_static(v.data_ptr(), self.num_tris, C.byref(self.desc),
                                                    self.buffer.data_ptr(), self.device_bytes, _stream(),
                                                    C.byref(h)), "hrpp_build_bvh_device_static")
            self.handle = h
            nn, nt, md = C.c_uint32(), C.c_uint32(), C.c_uint32()
            _check(lib.hrpp_bvh_info(h, C.byref(nn), C.byref(nt), C.byref(md)), "hrpp_bvh_info")
            self.num_nodes, self.max_depth = nn.value, md.value
            return self
        need = lib.hrpp_bvh_device_build_scratch_bytes(self.num_tris)
        if need == 0:
            raise HrppError("hrpp_bvh_device_build_scratch_bytes: no scratch size (bad count or no device)")
        self.device_bytes = lib.hrpp_bvh_required_bytes(self.num_tris, C.byref(self.desc))
        self._raw, self.buffer = _aligned(self.device_bytes, v.device)
        scratch_raw, scratch = _aligned(need, v.device)
        h = C.c_void_p()
        self.handle = None
        _check(lib.hrpp_build_bvh_device(v.data_ptr(), self.num_tris, C.byref(self.desc), scratch.data_ptr(), need,
                                         self.buffer.data_ptr(), self.device_bytes, _stream(), C.byref(h)),
               "hrpp_build_bvh_device")
        del scratch_raw, scratch
        self.handle = h
        nn, nt, md = C.c_uint32(), C.c_uint32(), C.c_uint32()
        _check(lib.hrpp_bvh_info(h, C.byref(nn), C.byref(nt), C.byref(md)), "hrpp_bvh_info")
        self.num_nodes, self.max_depth = nn.value, md.value
        return self

    def wide_info(self) -> dict:
        """The 4-wide tree of the plain-traversal baseline: nodes, root reference, stack need, depth."""
        n, r, k, d = C.c_uint32(), C.c_uint32(), C.c_uint32(), C.c_uint32()
        _check(load_library().hrpp_bvh_wide_info(self.handle, C.byref(n), C.byref(r), C.byref(k), C.byref(d)),
               "hrpp_bvh_wide_info")
        return dict(num_nodes=n.value, root_ref=r.value, stack_need=k.value, depth=d.value)

    def wide_export(self) -> np.ndarray:
        """The wide nodes as uint32 [nodes, 32] (layout in include/hrpp.h)."""
        m = self.wide_info()["num_nodes"]
        out = np.zeros((m, 32), np.uint32)
        _check(load_library().hrpp_bvh_wide_export(self.handle, out.ctypes.data if m else None, out.size),
               "hrpp_bvh_wide_export")
        return out

    def upload(self, device: str = "cuda"):
        self._raw, self.buffer = _aligned(self.device_bytes, device)
        _check(load_library().hrpp_bvh_upload(self.handle, self.buffer.data_ptr(), self.device_bytes, _stream()),
               "hrpp_bvh_upload")

    def export(self) -> dict:
        """Canonical depth-first tree as numpy arrays."""
        m, n = self.num_nodes, self.num_tris
        out = dict(box=np.zeros((m, 6), np.float32), right=np.zeros(m, np.uint32), first=np.zeros(m, np.uint32),
                   count=np.zeros(m, np.uint32), depth=np.zeros(m, np.uint32), perm=np.zeros(n, np.uint32))
        c = _Canon(out["box"].ctypes.data, out["right"].ctypes.data, out["first"].ctypes.data,
                   out["count"].ctypes.data, out["depth"].ctypes.data, out["perm"].ctypes.data)
        _check(load_library().hrpp_bvh_export(self.handle, C.byref(c)), "hrpp_bvh_export")
        return out

    def close(self):
        if getattr(self, "handle", None):
            load_library().hrpp_bvh_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Predictor:
    """A predictor table bound to one BVH (one per query type, hit-any / hit-all)."""

    def __init__(self, bvh: BVH, log2_entries: int = 12, ways: int = 4, origin_bits: int = 5, dir_bits: int = 6,
                 epoch_rays: int = 1 << 17, hash_mode: int = 0, go_up_level: int = 0, inline_lanes: int = 0,
                 replace_policy: int = 0, first_epoch_rays: int = 0, device: str = "cuda"):
        lib = load_library()
        self.desc = _PredDesc(log2_entries, ways, origin_bits, dir_bits, epoch_rays, hash_mode, go_up_level,
                              inline_lanes, replace_policy, first_epoch_rays)
        need = lib.hrpp_predictor_required_bytes(C.byref(self.desc))
        if need == 0:
            raise HrppError("hrpp_predictor_required_bytes: invalid descriptor")
        self.table_bytes = lib.hrpp_predictor_table_bytes(C.byref(self.desc))
        self.entry_bytes = 32 if ways <= 4 else 64
        self._raw, self.buffer = _aligned(need, device)
        h = C.c_void_p()
        _check(lib.hrpp_predictor_create(bvh.handle, C.byref(self.desc), self.buffer.data_ptr(), need, _stream(),
                                         C.byref(h)), "hrpp_predictor_create")
        self.handle = h
        self.bvh = bvh
        self.device_bytes = need

    @property
    def ways(self) -> int:
        return self.desc.ways

    def reset(self):
        _check(load_library().hrpp_predictor_reset(self.handle, _stream()), "hrpp_predictor_reset")

    def export_raw(self) -> np.ndarray:
        buf = np.empty(self.table_bytes, np.uint8)
        _check(load_library().hrpp_predictor_export(self.handle, buf.ctypes.data, buf.nbytes, _stream()),
               "hrpp_predictor_export")
        return buf

    def export(self):
        """(tags uint64 [N], slots uint32 [N, W]) of the current table."""
        raw = self.export_raw().reshape(-1, self.entry_bytes)
        tags = raw[:, 0:8].copy().view(np.uint64).reshape(-1)
        slots = raw[:, 8:8 + 4 * self.ways].copy().view(np.uint32).reshape(-1, self.ways)
        return tags, slots

    def import_raw(self, raw: np.ndarray):
        raw = np.ascontiguousarray(raw, np.uint8)
        _check(load_library().hrpp_predictor_import(self.handle, raw.ctypes.data, raw.nbytes, _stream()),
               "hrpp_predictor_import")

    def close(self):
        if getattr(self, "handle", None):
            load_library().hrpp_predictor_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def new_stats(device: str = "cuda") -> torch.Tensor:
    return torch.zeros(STATS_SLOTS, dtype=torch.int64, device=device)


def stats_dict(stats: torch.Tensor) -> dict:
    v = stats.detach().cpu().numpy().astype(np.uint64)
    return {k: int(v[i]) for i, k in enumerate(STAT_NAMES)}


def _rays_ok(rays: torch.Tensor):
    if not (rays.is_cuda and rays.dtype == torch.float32 and rays.dim() == 2 and rays.shape[1] == 8
            and rays.is_contiguous()):
        raise HrppError("rays must be a contiguous cuda float32 tensor of shape [n, 8]")


def trace_anyhit(bvh: BVH, pred: Predictor | None, rays: torch.Tensor, out: torch.Tensor | None = None,
                 stats: torch.Tensor | None = None) -> torch.Tensor:
    """Occlusion flags (uint8 [n]) for rays [n, 8]."""
    _rays_ok(rays)
    n = rays.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.uint8, device=rays.device)
    _check(load_library().hrpp_trace_anyhit(bvh.handle, pred.handle if pred is not None else None, rays.data_ptr(),
                                            n, out.data_ptr(), stats.data_ptr() if stats is not None else None,
                                            _stream()), "hrpp_trace_anyhit")
    return out


def trace_closest(bvh: BVH, pred: Predictor | None, rays: torch.Tensor, mode: str = "paper",
                  out: torch.Tensor | None = None, stats: torch.Tensor | None = None) -> torch.Tensor:
    """Closest hits as float32 [n, 4] (t, u, v, prim bits) for rays [n, 8]."""
    _rays_ok(rays)
    n = rays.shape[0]
    if out is None:
        out = torch.empty((n, 4), dtype=torch.float32, device=rays.device)
    _check(load_library().hrpp_trace_closest(bvh.handle, pred.handle if pred is not None else None,
                                             rays.data_ptr(), n, CLOSEST_MODES[mode], out.data_ptr(),
                                             stats.data_ptr() if stats is not None else None, _stream()),
           "hrpp_trace_closest")
    return out


def trace_wide_anyhit(bvh: BVH, rays: torch.Tensor, out: torch.Tensor | None = None,
                      stats: torch.Tensor | None = None) -> torch.Tensor:
    """Any-hit flags from plain traversal of the 4-wide tree (the baseline)."""
    _rays_ok(rays)
    n = rays.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.uint8, device=rays.device)
    _check(load_library().hrpp_trace_wide_anyhit(bvh.handle, rays.data_ptr(), n, out.data_ptr(),
                                                 stats.data_ptr() if stats is not None else None, _stream()),
           "hrpp_trace_wide_anyhit")
    return out


def trace_wide_closest(bvh: BVH, rays: torch.Tensor, out: torch.Tensor | None = None,
                       stats: torch.Tensor | None = None) -> torch.Tensor:
    """Exact closest hits from plain traversal of the 4-wide tree (the baseline)."""
    _rays_ok(rays)
    n = rays.shape[0]
    if out is None:
        out = torch.empty((n, 4), dtype=torch.float32, device=rays.device)
    _check(load_library().hrpp_trace_wide_closest(bvh.handle, rays.data_ptr(), n, out.data_ptr(),
                                                  stats.data_ptr() if stats is not None else None, _stream()),
           "hrpp_trace_wide_closest")
    return out


def get_error(bvh: BVH | None = None):
    _check(load_library().hrpp_get_error(bvh.handle if bvh is not None else None, _stream()), "hrpp_get_error")


def profile_start():
    """Start per-kernel event timing inside the library."""
    _check(load_library().hrpp_profile_start(), "hrpp_profile_start")


TOUCH_REGIONS = ("nodes", "tris", "leafbox", "entries", "cnode")
TOUCH_KINDS = ("k_predict", "k_epoch_empty", "k_traverse_queue", "k_traverse_plain")


def profile_touch(bvh: BVH | None, pred: Predictor | None = None):
    """Mark the 128-byte lines that counting traces on (bvh, pred) touch (measurement only).

    Returns a reader: read() gives {kernel kind: {region: distinct lines}} of the traces since the
    last read and clears the bitmap.  profile_touch(None) stops the marking."""
    lib = load_library()
    if bvh is None:
        _check(lib.hrpp_profile_touch(None, None, None, 0, None), "hrpp_profile_touch")
        return None
    layout = (C.c_uint32 * 11)()
    ph = pred.handle if pred is not None else None
    _check(lib.hrpp_profile_touch(bvh.handle, ph, None, 0, layout), "hrpp_profile_touch")
    block = int(layout[0])
    bits = torch.zeros(len(TOUCH_KINDS) * block, dtype=torch.int32, device="cuda")
    _check(lib.hrpp_profile_touch(bvh.handle, ph, bits.data_ptr(), bits.numel(), layout), "hrpp_profile_touch")
    offs = [int(layout[1 + r]) for r in range(len(TOUCH_REGIONS))]
    lines = [int(layout[6 + r]) for r in range(len(TOUCH_REGIONS))]

    def read() -> dict:
        torch.cuda.synchronize()
        words = bits.cpu().numpy().view(np.uint32).reshape(len(TOUCH_KINDS), block)
        bits.zero_()
        out = {}
        for k, kind in enumerate(TOUCH_KINDS):
            out[kind] = {}
            for r, reg in enumerate(TOUCH_REGIONS):
                w = words[k, offs[r]: offs[r] + (lines[r] + 31) // 32]
                out[kind][reg] = int(np.unpackbits(w.view(np.uint8)).sum())
        return out
    return read


def profile_stop() -> dict:
    """Stop timing; returns {kernel name: (launches, total ms)}."""
    arr = (_KernelTime * 16)()
    n = C.c_uint32()
    _check(load_library().hrpp_profile_stop(arr, 16, C.byref(n)), "hrpp_profile_stop")
    return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms)) for i in range(min(n.value, 16))}


class Batch:
    """Many independent traces launched together (optionally as one hipGraph).

    ``jobs``: dicts with keys bvh, pred (or None), rays (cuda float32 [n, 8]),
    query ("any" | "closest"), mode ("paper" | "exact"), out (optional), stats
    (optional int64 [32] cuda tensor).  Outputs are allocated if not given and
    are available as ``batch.outputs[i]``.
    """

    def __init__(self, jobs, device: str = "cuda"):
        lib = load_library()
        self._keep = []
        arr = (_BatchJob * len(jobs))()
        self.outputs = []
        for i, j in enumerate(jobs):
            rays = j["rays"]
            _rays_ok(rays)
            n = rays.shape[0]
            query = j.get("query", "any")
            out = j.get("out")
            if out is None:
                out = (torch.empty(n, dtype=torch.uint8, device=rays.device) if query == "any"
                       else torch.empty((n, 4), dtype=torch.float32, device=rays.device))
            st = j.get("stats")
            pred = j.get("pred")
            arr[i] = _BatchJob(j["bvh"].handle, pred.handle if pred is not None else None, rays.data_ptr(), n,
                               0 if query == "any" else 1, CLOSEST_MODES[j.get("mode", "paper")], out.data_ptr(),
                               st.data_ptr() if st is not None else None)
            self._keep += [rays, out, st, j["bvh"], pred]
            self.outputs.append(out)
        need = lib.hrpp_batch_required_bytes(len(jobs))
        self._raw, self.buffer = _aligned(need, device)
        h = C.c_void_p()
        _check(lib.hrpp_batch_create(arr, len(jobs), self.buffer.data_ptr(), need, _stream(), C.byref(h)),
               "hrpp_batch_create")
        self.handle = h

    def launch(self, use_graph: bool = True):
        _check(load_library().hrpp_batch_launch(self.handle, 1 if use_graph else 0, _stream()), "hrpp_batch_launch")

    def close(self):
        if getattr(self, "handle", None):
            load_library().hrpp_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching request server over resident scenes.

    ``scenes``: list of (bvh, [any-hit predictors], [closest-hit predictors]).
    ``pool_bytes``: device budget for in-flight request rays and results.
    Requests carry host tensors (pinned for asynchronous copies): rays
    float32 [n, 8]; results uint8 [n] (query "any") or float32 [n, 4]
    (query "closest", exact closest hit).
    """

    def __init__(self, scenes, slots: int = 8, pool_bytes: int = 1 << 30, device: str = "cuda"):
        lib = load_library()
        self._keep = []
        arr = (_ServeScene * len(scenes))()
        for i, (bvh, anyp, clp) in enumerate(scenes):
            a = (C.c_void_p * len(anyp))(*[p.handle.value for p in anyp])
            c = (C.c_void_p * len(clp))(*[p.handle.value for p in clp])
            self._keep += [a, c, bvh, list(anyp), list(clp)]
            arr[i] = _ServeScene(bvh.handle, C.cast(a, C.c_void_p), len(anyp), C.cast(c, C.c_void_p), len(clp))
        self._raw, self.pool = _aligned(pool_bytes, device)
        torch.cuda.synchronize()
        h = C.c_void_p()
        _check(lib.hrpp_serve_create(arr, len(scenes), slots, self.pool.data_ptr(), pool_bytes, C.byref(h)),
               "hrpp_serve_create")
        self.handle = h
        self._reqs = {}

    def add_scene(self, bvh: BVH, any_preds, closest_preds) -> int:
        """Add a scene while the server runs; returns its index for submit."""
        a = (C.c_void_p * len(any_preds))(*[p.handle.value for p in any_preds])
        c = (C.c_void_p * len(closest_preds))(*[p.handle.value for p in closest_preds])
        self._keep += [a, c, bvh, list(any_preds), list(closest_preds)]
        sc = _ServeScene(bvh.handle, C.cast(a, C.c_void_p), len(any_preds), C.cast(c, C.c_void_p),
                         len(closest_preds))
        torch.cuda.current_stream().synchronize()     # the predictors' creation (reset) has run
        idx = C.c_uint32()
        _check(load_library().hrpp_serve_add_scene(self.handle, C.byref(sc), C.byref(idx)), "hrpp_serve_add_scene")
        return idx.value

    def remove_scene(self, index: int):
        """Refuse new requests for a scene and wait for its queued and running ones."""
        _check(load_library().hrpp_serve_remove_scene(self.handle, index), "hrpp_serve_remove_scene")

    def submit(self, scene: int, query: str, rays: torch.Tensor, out: torch.Tensor) -> int:
        if rays.is_cuda or out.is_cuda or not rays.is_contiguous() or not out.is_contiguous():
            raise HrppError("serving requests use contiguous host tensors")
        rid = C.c_uint64()
        _check(load_library().hrpp_serve_submit(self.handle, scene, 0 if query == "any" else 1, rays.data_ptr(),
                                                rays.shape[0], out.data_ptr(), C.byref(rid)), "hrpp_serve_submit")
        self._reqs[rid.value] = (rays, out)
        return rid.value

    def poll(self, rid: int) -> dict:
        """State and timings of a request; the poll that reports it done (state 2) retires it."""
        info = _RequestInfo()
        _check(load_library().hrpp_serve_poll(self.handle, rid, C.byref(info)), "hrpp_serve_poll")
        if info.state == 2:
            self._reqs.pop(rid, None)
        return dict(state=info.state, status=info.status, queue_ms=info.queue_ms, service_ms=info.service_ms,
                    latency_ms=info.latency_ms)

    def held(self) -> int:
        """Request records the server holds (queued, running, or done and not yet polled)."""
        v = C.c_uint64()
        _check(load_library().hrpp_serve_held(self.handle, C.byref(v)), "hrpp_serve_held")
        return v.value

    def wait_all(self):
        _check(load_library().hrpp_serve_wait_all(self.handle), "hrpp_serve_wait_all")

    def pool_peak(self) -> int:
        v = C.c_size_t()
        _check(load_library().hrpp_serve_pool_peak(self.handle, C.byref(v)), "hrpp_serve_pool_peak")
        return v.value

    def close(self):
        if getattr(self, "handle", None):
            load_library().hrpp_serve_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
