"""Seeded synthetic scenes and rays for the HRPP workloads.

This module is shared input plumbing: both the CPU oracle's tests and the GPU
library's tests/benchmarks draw their inputs from here.  It holds none of the
method's arithmetic (no hashing, no BVH, no ray-box or ray-triangle test):
it only produces triangle soups, heightfields, cameras and ray arrays with
numpy's PCG64 generator.

Conventions
-----------
* Triangles: float32 array ``[n, 3, 3]`` (vertex, xyz).  The primitive id of a
  triangle is its row index.
* Rays: float32 array ``[n, 8]`` laid out as ``ox oy oz tmin dx dy dz tmax``
  (32 bytes per ray).
* Hits (input to the secondary-ray builders): float32 ``t`` and uint32
  ``prim`` arrays; ``prim == 0xFFFFFFFF`` means a miss.

The paper's own scenes (PBRT's Teapot ... Sportscar) are not available; the
generators below are the stand-ins, with sizes chosen to match the paper's
scale (a one-million-triangle scene, like its Buddha) and its 8 samples per
pixel (AO rays per primary hit).
"""
from __future__ import annotations

import math
import numpy as np

MISS = np.uint32(0xFFFFFFFF)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ---------------------------------------------------------------------------
# Scenes
# ---------------------------------------------------------------------------

def triangle_soup(seed: int, n: int, edge: float = 0.05) -> np.ndarray:
    """``n`` near-equilateral triangles scattered in the unit cube.

    Centroid uniform in [0,1]^3, edge ``edge * U[0.8, 1.2]``, plane normal
    uniform on the sphere, in-plane rotation uniform in [0, 2pi).
    """
    g = rng(seed)
    c = g.random((n, 3))
    e = edge * g.uniform(0.8, 1.2, n)
    nz = g.uniform(-1.0, 1.0, n)
    phi = g.uniform(0.0, 2 * np.pi, n)
    r = np.sqrt(np.maximum(0.0, 1.0 - nz * nz))
    nrm = np.stack([r * np.cos(phi), r * np.sin(phi), nz], axis=1)
    # orthonormal tangent frame (any helper vector not parallel to the normal)
    helper = np.where(np.abs(nrm[:, :1]) < 0.9, np.array([[1.0, 0, 0]]), np.array([[0, 1.0, 0]]))
    t1 = np.cross(nrm, helper)
    t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
    t2 = np.cross(nrm, t1)
    ang = g.uniform(0.0, 2 * np.pi, n)
    rad = e / np.sqrt(3.0)  # circumradius of an equilateral triangle
    verts = np.empty((n, 3, 3))
    for k in range(3):
        a = ang + k * (2 * np.pi / 3)
        verts[:, k, :] = c + rad[:, None] * (np.cos(a)[:, None] * t1 + np.sin(a)[:, None] * t2)
    return verts.astype(np.float32)


def _value_noise_fbm(g: np.random.Generator, x: np.ndarray, z: np.ndarray,
                     octaves: int = 6, lacunarity: float = 2.0, gain: float = 0.5,
                     base_freq: float = 4.0) -> np.ndarray:
    """Fractal sum of value noise on [0,1]^2, normalised to [-1, 1]."""
    total = np.zeros_like(x, dtype=np.float64)
    amp, freq, norm = 1.0, base_freq, 0.0
    for _ in range(octaves):
        res = int(math.ceil(freq)) + 2
        lattice = g.uniform(-1.0, 1.0, (res, res))
        fx, fz = x * freq, z * freq
        ix, iz = np.floor(fx).astype(np.int64), np.floor(fz).astype(np.int64)
        tx, tz = fx - ix, fz - iz
        sx, sz = tx * tx * (3 - 2 * tx), tz * tz * (3 - 2 * tz)  # smoothstep
        v00 = lattice[ix, iz]
        v10 = lattice[ix + 1, iz]
        v01 = lattice[ix, iz + 1]
        v11 = lattice[ix + 1, iz + 1]
        a = v00 + (v10 - v00) * sx
        b = v01 + (v11 - v01) * sx
        total += amp * (a + (b - a) * sz)
        norm += amp
        amp *= gain
        freq *= lacunarity
    return total / norm


class Heightfield:
    """A noise heightfield over [0,1]^2 in (x, z), y = amplitude * fBm."""

    def __init__(self, seed: int, amplitude: float = 0.1):
        self.seed = seed
        self.amplitude = amplitude
        # draw all octave lattices up front so height() is a pure function
        self._g_state = rng(seed).bit_generator.state

    def height(self, x: np.ndarray, z: np.ndarray) -> np.ndarray:
        g = np.random.Generator(np.random.PCG64())
        g.bit_generator.state = self._g_state
        return self.amplitude * _value_noise_fbm(g, np.asarray(x, np.float64), np.asarray(z, np.float64))

    def triangles(self, side: int) -> np.ndarray:
        """``side x side`` vertex grid, quads split on the (0,0)-(1,1) diagonal, row-major."""
        u = np.linspace(0.0, 1.0, side)
        X, Z = np.meshgrid(u, u, indexing="ij")      # X[i, j] = u[i], Z[i, j] = u[j]
        Y = self.height(X, Z)
        V = np.stack([X, Y, Z], axis=-1)             # [side, side, 3]
        v00 = V[:-1, :-1].reshape(-1, 3)
        v10 = V[1:, :-1].reshape(-1, 3)
        v01 = V[:-1, 1:].reshape(-1, 3)
        v11 = V[1:, 1:].reshape(-1, 3)
        # quad q -> triangles 2q (v00, v10, v11) and 2q+1 (v00, v11, v01)
        t = np.empty((v00.shape[0] * 2, 3, 3))
        t[0::2, 0], t[0::2, 1], t[0::2, 2] = v00, v10, v11
        t[1::2, 0], t[1::2, 1], t[1::2, 2] = v00, v11, v01
        return t.astype(np.float32)


def _cube_triangles(lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    """12 triangles of axis-aligned boxes [lo, hi] (arrays [m, 3])."""
    m = lo.shape[0]
    corners = np.empty((m, 8, 3))
    for k in range(8):
        corners[:, k, 0] = np.where(k & 1, hi[:, 0], lo[:, 0])
        corners[:, k, 1] = np.where(k & 2, hi[:, 1], lo[:, 1])
        corners[:, k, 2] = np.where(k & 4, hi[:, 2], lo[:, 2])
    faces = [(0, 2, 6, 4), (1, 5, 7, 3),   # x = lo, x = hi
             (0, 4, 5, 1), (2, 3, 7, 6),   # y = lo, y = hi
             (0, 1, 3, 2), (4, 6, 7, 5)]   # z = lo, z = hi
    out = np.empty((m, 12, 3, 3))
    for f, (a, b, c, d) in enumerate(faces):
        out[:, 2 * f, 0], out[:, 2 * f, 1], out[:, 2 * f, 2] = corners[:, a], corners[:, b], corners[:, c]
        out[:, 2 * f + 1, 0], out[:, 2 * f + 1, 1], out[:, 2 * f + 1, 2] = corners[:, a], corners[:, c], corners[:, d]
    return out.reshape(m * 12, 3, 3)


def terrain_scene(seed: int = 2, side: int = 724, n_boxes: int = 4096,
                  total: int = 1 << 20, amplitude: float = 0.1):
    """The one-million-triangle test scene: heightfield plus boxes sitting on it.

    Returns ``(tris, heightfield)``.  The first ``total - 12 * n_boxes``
    heightfield triangles (row-major) are kept, then all box triangles, so the
    count is exactly ``total``.
    """
    hf = Heightfield(seed, amplitude)
    ht = hf.triangles(side)
    g = rng(seed + 1000)
    s = g.uniform(0.005, 0.05, n_boxes)
    cx, cz = g.random(n_boxes), g.random(n_boxes)
    base = hf.height(cx, cz)
    lo = np.stack([cx - s / 2, base, cz - s / 2], axis=1)
    hi = np.stack([cx + s / 2, base + s, cz + s / 2], axis=1)
    bt = _cube_triangles(lo, hi).astype(np.float32)
    keep = total - bt.shape[0]
    if keep > ht.shape[0] or keep < 0:
        raise ValueError("heightfield too small for the requested total")
    return np.concatenate([ht[:keep], bt], axis=0), hf


def scaled_terrain_scene(seed: int, total: int, amplitude: float = 0.1):
    """A smaller copy of :func:`terrain_scene` (same recipe, ~``total`` triangles)."""
    n_boxes = max(1, total // 256)
    side = int(math.ceil(math.sqrt((total - 12 * n_boxes) / 2.0))) + 2
    return terrain_scene(seed, side=side, n_boxes=n_boxes, total=total, amplitude=amplitude)


# ---------------------------------------------------------------------------
# Rays
# ---------------------------------------------------------------------------

def pack_rays(o: np.ndarray, d: np.ndarray, tmin, tmax) -> np.ndarray:
    n = o.shape[0]
    r = np.empty((n, 8), np.float32)
    r[:, 0:3] = o
    r[:, 3] = tmin
    r[:, 4:7] = d
    r[:, 7] = tmax
    return r


def tiny_shadow_rays(seed: int = 1, n: int = 4096) -> np.ndarray:
    """Shadow rays from the floor y=0 to a 0.2x0.2 area light at y=1.5.

    Direction unnormalised (target - origin), interval (0, 1).
    """
    g = rng(seed + 7)
    o = np.stack([g.random(n), np.zeros(n), g.random(n)], axis=1)
    tgt = np.stack([0.5 + g.uniform(-0.1, 0.1, n), np.full(n, 1.5), 0.5 + g.uniform(-0.1, 0.1, n)], axis=1)
    o32 = o.astype(np.float32)
    d32 = (tgt.astype(np.float32) - o32).astype(np.float32)
    return pack_rays(o32, d32, 0.0, 1.0)


BAYER4 = np.array([[0, 8, 2, 10], [12, 4, 14, 6], [3, 11, 1, 9], [15, 7, 13, 5]])


def pixel_order(width: int, height: int, order: str = "bayer") -> np.ndarray:
    """Pixel linear ids (y * width + x) in trace order.

    ``bayer``: 16 interleaved passes; pass j holds the pixels whose
    (x mod 4, y mod 4) cell has Bayer rank j; row-major within a pass.
    ``rowmajor``: plain row-major.
    """
    ids = np.arange(width * height)
    if order == "rowmajor":
        return ids
    x, y = ids % width, ids // width
    rank = BAYER4[y % 4, x % 4]
    return ids[np.argsort(rank, kind="stable")]


class Camera:
    def __init__(self, eye=(0.5, 0.5, 0.3), look=(0.5, 0.0, 0.5), up=(0.0, 1.0, 0.0),
                 vfov_deg: float = 40.0, width: int = 1920, height: int = 1080):
        self.eye = np.asarray(eye, np.float64)
        self.look = np.asarray(look, np.float64)
        self.up = np.asarray(up, np.float64)
        self.vfov = vfov_deg
        self.width, self.height = width, height

    def rays(self, order: str = "bayer", offset=(0.5, 0.5)):
        """Unit-direction primary rays through one sample position per pixel
        (``offset`` within the pixel, (0.5, 0.5) = the centre), interval (0, inf).

        Returns ``(rays, pixel_ids)`` with rays in trace order.
        """
        w = self.look - self.eye
        w /= np.linalg.norm(w)
        u = np.cross(w, self.up)
        u /= np.linalg.norm(u)
        v = np.cross(u, w)
        th = math.tan(math.radians(self.vfov) / 2)
        aspect = self.width / self.height
        pid = pixel_order(self.width, self.height, order)
        px, py = pid % self.width, pid // self.width
        sx = (2 * (px + offset[0]) / self.width - 1) * th * aspect
        sy = (1 - 2 * (py + offset[1]) / self.height) * th
        d = w[None, :] + sx[:, None] * u[None, :] + sy[:, None] * v[None, :]
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        o = np.broadcast_to(self.eye, d.shape)
        return pack_rays(o.astype(np.float32), d.astype(np.float32), 0.0, np.inf), pid

    def assert_all_hit_terrain(self, rays: np.ndarray, amplitude: float) -> None:
        """Check, without tracing, that every ray must hit the heightfield.

        A descending ray that crosses y = +amp and y = -amp inside the
        footprint [0,1]^2 crosses the continuous surface in between.
        """
        o, d = rays[:, 0:3].astype(np.float64), rays[:, 4:7].astype(np.float64)
        if np.any(d[:, 1] >= 0):
            raise AssertionError("a primary ray does not descend")
        for yplane in (amplitude, -amplitude):
            t = (yplane - o[:, 1]) / d[:, 1]
            p = o + t[:, None] * d
            if np.any((p[:, 0] < 0) | (p[:, 0] > 1) | (p[:, 2] < 0) | (p[:, 2] > 1)):
                raise AssertionError("a primary ray leaves the terrain footprint")


def _face_normals(tris: np.ndarray, prim: np.ndarray) -> np.ndarray:
    t = tris[prim].astype(np.float64)
    n = np.cross(t[:, 1] - t[:, 0], t[:, 2] - t[:, 0])
    return n / np.linalg.norm(n, axis=1, keepdims=True)


def _hit_frame(tris, rays, t, prim, eps):
    """Offset hit points and facing normals; rows of missed primaries are
    returned with ``ok = False`` (their secondary rays are made invalid)."""
    ok = prim != MISS
    safe = np.where(ok, prim, 0)
    tt = np.where(ok, t, 0.0).astype(np.float64)
    o, d = rays[:, 0:3].astype(np.float64), rays[:, 4:7].astype(np.float64)
    p = o + tt[:, None] * d
    n = _face_normals(tris, safe)
    facing = np.where((np.sum(n * d, axis=1) < 0)[:, None], n, -n)
    return p + eps * facing, facing, ok


def shadow_rays_from_hits(tris, rays, t, prim, seed: int, light_center=(0.5, 1.0, 0.5),
                          light_size: float = 0.1, eps: float = 1e-4) -> np.ndarray:
    """One shadow ray per hit point towards a square area light (y = const).

    Origin offset by ``eps`` along the normal facing the incoming ray;
    direction = light sample - origin (unnormalised); interval (0, 1).  A
    primary ray that missed (a binary32 crack between triangles can let a
    ray through) yields an invalid ray (zero direction).
    """
    o, _, ok = _hit_frame(tris, rays, t, prim, eps)
    g = rng(seed + 11)
    n = o.shape[0]
    lc = np.asarray(light_center, np.float64)
    s = np.stack([lc[0] + light_size * g.uniform(-0.5, 0.5, n), np.full(n, lc[1]),
                  lc[2] + light_size * g.uniform(-0.5, 0.5, n)], axis=1)
    o32 = o.astype(np.float32)
    d32 = (s.astype(np.float32) - o32).astype(np.float32)
    d32[~ok] = 0.0
    return pack_rays(o32, d32, 0.0, 1.0)


def _concentric_disk(u1, u2):
    """Shirley-Chiu concentric square-to-disk map."""
    a, b = 2 * u1 - 1, 2 * u2 - 1
    r = np.where(np.abs(a) > np.abs(b), a, b)
    with np.errstate(divide="ignore", invalid="ignore"):
        phi = np.where(np.abs(a) > np.abs(b), (np.pi / 4) * (b / a), np.pi / 2 - (np.pi / 4) * (a / b))
    phi = np.where((a == 0) & (b == 0), 0.0, phi)
    return r * np.cos(phi), r * np.sin(phi)


def _onb(n):
    """Branchless orthonormal basis (Duff et al. 2017) around unit normals."""
    s = np.where(n[:, 2] >= 0, 1.0, -1.0)
    a = -1.0 / (s + n[:, 2])
    b = n[:, 0] * n[:, 1] * a
    t1 = np.stack([1 + s * n[:, 0] * n[:, 0] * a, s * b, -s * n[:, 0]], axis=1)
    t2 = np.stack([b, s + n[:, 1] * n[:, 1] * a, -n[:, 1]], axis=1)
    return t1, t2


def ao_rays_from_hits(tris, rays, t, prim, seed: int, samples: int = 8, tmax: float = 0.05,
                      eps: float = 1e-4) -> np.ndarray:
    """``samples`` cosine-weighted hemisphere rays per hit, sample-major order.

    Unit directions about the facing normal; interval (0, tmax).  Rays of
    missed primaries are invalid (zero direction).
    """
    o, nf, ok = _hit_frame(tris, rays, t, prim, eps)
    t1, t2 = _onb(nf)
    g = rng(seed + 13)
    m = o.shape[0]
    out = []
    for _ in range(samples):
        x, y = _concentric_disk(g.random(m), g.random(m))
        z = np.sqrt(np.maximum(0.0, 1 - x * x - y * y))
        d = x[:, None] * t1 + y[:, None] * t2 + z[:, None] * nf
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        d[~ok] = 0.0
        out.append(pack_rays(o.astype(np.float32), d.astype(np.float32), 0.0, tmax))
    return np.concatenate(out, axis=0)


def surface_points(tris: np.ndarray, count: int, seed: int):
    """Points sampled uniformly by area on ``tris`` with their unit normals."""
    g = rng(seed)
    t = tris.astype(np.float64)
    area = 0.5 * np.linalg.norm(np.cross(t[:, 1] - t[:, 0], t[:, 2] - t[:, 0]), axis=1)
    cdf = np.cumsum(area)
    pick = np.searchsorted(cdf, g.random(count) * cdf[-1], side="right")
    pick = np.minimum(pick, t.shape[0] - 1)
    r1, r2 = np.sqrt(g.random(count)), g.random(count)
    a, b = 1 - r1, r1 * (1 - r2)
    tt = t[pick]
    p = a[:, None] * tt[:, 0] + b[:, None] * tt[:, 1] + (1 - a - b)[:, None] * tt[:, 2]
    n = np.cross(tt[:, 1] - tt[:, 0], tt[:, 2] - tt[:, 0])
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    return p, n


def scene_diagonal(tris: np.ndarray) -> float:
    v = tris.reshape(-1, 3).astype(np.float64)
    return float(np.linalg.norm(v.max(0) - v.min(0)))


# ---------------------------------------------------------------------------
# Named workloads (sizes of the benchmark configurations)
# ---------------------------------------------------------------------------

TINY = dict(seed=1, n_tris=256, n_rays=4096, log2_entries=12, ways=4, origin_bits=5, dir_bits=6, epoch=256)
AT_SCALE = dict(seed=2, width=1920, height=1080, log2_entries=20, ways=8, origin_bits=5, dir_bits=6,
                epoch=1 << 19, light_center=(0.5, 1.0, 0.5), light_size=0.1,
                # (origin bits, direction bits, epoch rays, inline lanes, first epoch
                # rays) of the hit-all and hit-any predictors, chosen by the autotuner
                # (table fixed at 2^20 x 8) and a sweep of the two-stream step: a first
                # epoch of one Bayer pass (2^17 rays, the whole view at 1/16 density)
                # for the hit-all predictor and four (2^19 rays) for the hit-any one,
                # then the rest of the frame in one epoch
                primary_q=(5, 7, 1 << 21, 1, 1 << 17), shadow_q=(6, 3, 1 << 21, 1, 1 << 19),
                # SAH leaves of at most 2 triangles (a terrain quad): on this scene leaves
                # of up to 4 straddle cells, and plain and HRPP traversal both run faster
                # with leaves of 2 (measured at leaf sizes 1 to 4)
                leaf_max=2,
                # two passes of treelet restructuring after the SAH build: the sum of
                # interior half areas falls from 151 to 128 and the two-stream step
                # runs faster over the restructured tree, plain and HRPP alike
                treelet_passes=2)
# the AO predictor: q_o 6, q_d 5, epochs of 2^22 rays (the largest; 7,372,800 rays
# make two), waves with >= 16 failing lanes traverse in place; a table of 2^16 x 8
# entries (4 MB), which stays in the last-level cache: the randomly addressed
# lookups of short incoherent rays missed it at 2^20 (64 MB), and a sweep of
# 2^16 .. 2^20 entries ran fastest at the smallest.  With the 2^20 table a short
# first epoch (2^16 rays) paid off; with 2^16 entries, which predict fewer rays,
# the schedule with the fewest epochs runs fastest (a sweep of first epochs 0 and
# 2^16 .. 2^18, epochs 2^21 and 2^22, in-place thresholds 1, 16, 32)
INCOHERENT = dict(seed=3, width=1280, height=720, samples=8, log2_entries=16, ways=8, origin_bits=6,
                  dir_bits=5, epoch=1 << 22, inline_lanes=16, first_epoch=0, tmax_frac=0.05)


def tiny_workload():
    """256-triangle soup and 4,096 shadow rays to an area light."""
    w = TINY
    return triangle_soup(w["seed"], w["n_tris"]), tiny_shadow_rays(w["seed"], w["n_rays"])


def camera_for(width: int, height: int) -> Camera:
    return Camera(width=width, height=height)


def terrain_workload(total: int = 1 << 20, width: int = 1920, height: int = 1080, seed: int = 2,
                     order: str = "bayer", offset=(0.5, 0.5)):
    """Scene and primary rays of the at-scale workload (optionally scaled
    down; ``offset`` = sample position within each pixel)."""
    if total == 1 << 20:
        tris, hf = terrain_scene(seed)
    else:
        tris, hf = scaled_terrain_scene(seed, total)
    cam = camera_for(width, height)
    rays, pid = cam.rays(order, offset)
    cam.assert_all_hit_terrain(rays, hf.amplitude)
    return tris, rays


# sample positions of the progressive frames (a 2 x 2 stratified pattern)
PROGRESSIVE_OFFSETS = ((0.25, 0.25), (0.75, 0.25), (0.25, 0.75), (0.75, 0.75))


def progressive_primaries(width: int = 1920, height: int = 1080, order: str = "bayer"):
    """Primary rays of the at-scale camera for each progressive frame."""
    cam = camera_for(width, height)
    return [cam.rays(order, off)[0] for off in PROGRESSIVE_OFFSETS]


# ---------------------------------------------------------------------------
# Many scenes (batching and serving workloads)
# ---------------------------------------------------------------------------

def soup_scene(seed: int, n: int) -> np.ndarray:
    """A random-triangle soup of n triangles with edge ~0.8 n^(-1/3) in the unit cube."""
    return triangle_soup(seed, n, edge=0.8 * n ** (-1.0 / 3.0))


def heightfield_scene(seed: int, n: int) -> np.ndarray:
    """A noise heightfield on a (floor(sqrt(n/2)) + 2)^2 vertex grid, trimmed to exactly n triangles."""
    side = int(math.floor(math.sqrt(n / 2.0))) + 2
    t = Heightfield(seed).triangles(side)
    return np.ascontiguousarray(t[:n])


def mixed_scene(seed: int, n: int) -> np.ndarray:
    """Soup or heightfield with probability 1/2 each (decided by the seed)."""
    return soup_scene(seed, n) if rng(seed).random() < 0.5 else heightfield_scene(seed, n)


def secondary_rays_on_surface(tris: np.ndarray, count: int, seed: int, shadow_fraction: float = 0.6,
                              ao_tmax_frac: float = 0.05, light_center=None, light_size: float = 0.2):
    """Shadow (to an area light above the scene) and AO (cosine hemisphere)
    rays from points sampled uniformly by area on the scene's triangles."""
    p, n = surface_points(tris, count, seed)
    g = rng(seed + 17)
    v = tris.reshape(-1, 3).astype(np.float64)
    lo, hi = v.min(0), v.max(0)
    diag = float(np.linalg.norm(hi - lo))
    ns = int(round(shadow_fraction * count))
    # face the normal towards +y (the light) for shadow rays; random side for AO
    up = np.where((n[:, 1] < 0)[:, None], -n, n)
    o = p + 1e-4 * diag * up
    lc = np.asarray(light_center if light_center is not None else [(lo[0] + hi[0]) / 2, hi[1] + 0.5 * diag,
                                                                    (lo[2] + hi[2]) / 2])
    s = np.stack([lc[0] + light_size * diag * g.uniform(-0.5, 0.5, ns), np.full(ns, lc[1]),
                  lc[2] + light_size * diag * g.uniform(-0.5, 0.5, ns)], 1)
    shadow = pack_rays(o[:ns].astype(np.float32), (s.astype(np.float32) - o[:ns].astype(np.float32)), 0.0, 1.0)
    m = count - ns
    t1, t2 = _onb(up[ns:])
    x, y = _concentric_disk(g.random(m), g.random(m))
    z = np.sqrt(np.maximum(0.0, 1 - x * x - y * y))
    d = x[:, None] * t1 + y[:, None] * t2 + z[:, None] * up[ns:]
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    ao = pack_rays(o[ns:].astype(np.float32), d.astype(np.float32), 0.0, ao_tmax_frac * diag)
    return shadow, ao


def log_uniform_int(g: np.random.Generator, lo: float, hi: float) -> int:
    return int(round(math.exp(g.uniform(math.log(lo), math.log(hi)))))
