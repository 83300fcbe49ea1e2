"""Independent fp64 geometry used by the pins (linear-algebra formulation).

Ray-triangle: solve o + t d = v0 + u e1 + v e2 as a 3x3 linear system with
numpy (not the Moller-Trumbore operation sequence).  Used to pin the binary32
code from outside and to find rays that pass within 1e-6 of a triangle edge,
where binary32 decisions may legitimately differ from exact ones.
"""
from __future__ import annotations

import numpy as np

EDGE_EPS = 1e-6


def solve_tuv(tris: np.ndarray, rays: np.ndarray):
    """All-pairs fp64 (t, u, v) and a validity mask; shapes [R, T]."""
    tr = np.asarray(tris, np.float64).reshape(-1, 3, 3)
    ry = np.asarray(rays, np.float64).reshape(-1, 8)
    v0 = tr[:, 0][None]                       # [1, T, 3]
    e1 = (tr[:, 1] - tr[:, 0])[None]
    e2 = (tr[:, 2] - tr[:, 0])[None]
    o = ry[:, None, 0:3]
    d = ry[:, None, 4:7]
    rhs = o - v0                              # [R, T, 3]
    dd = np.broadcast_to(-d, rhs.shape)
    ee1 = np.broadcast_to(e1, rhs.shape)
    ee2 = np.broadcast_to(e2, rhs.shape)
    A = np.stack([dd, ee1, ee2], axis=-1)     # columns: -d, e1, e2
    det = np.linalg.det(A)
    ok = np.abs(det) > 1e-300
    A_safe = np.where(ok[..., None, None], A, np.eye(3))
    sol = np.linalg.solve(A_safe, rhs[..., None])[..., 0]
    return sol[..., 0], sol[..., 1], sol[..., 2], ok


def near_edge(tris: np.ndarray, rays: np.ndarray, eps: float = EDGE_EPS) -> np.ndarray:
    """Per ray: True if some triangle's fp64 solution lies within eps of its
    boundary (an edge, or the interval ends tmin/tmax) while not clearly outside."""
    t, u, v, ok = solve_tuv(tris, rays)
    ry = np.asarray(rays, np.float64).reshape(-1, 8)
    w = 1.0 - u - v
    m = np.minimum(np.minimum(u, v), w)
    tmin, tmax = ry[:, 3:4], ry[:, 7:8]
    scale = np.maximum(1.0, np.abs(t))
    edge = ok & (np.abs(m) <= eps) & (t > tmin - eps * scale) & (t < tmax + eps * scale)
    inside = ok & (m >= -eps)
    interval = inside & ((np.abs(t - tmin) <= eps * scale) | (np.abs(t - tmax) <= eps * scale))
    degenerate = ~ok | (np.abs(np.linalg.norm(np.cross(
        np.asarray(tris, np.float64).reshape(-1, 3, 3)[:, 1] - np.asarray(tris, np.float64).reshape(-1, 3, 3)[:, 0],
        np.asarray(tris, np.float64).reshape(-1, 3, 3)[:, 2] - np.asarray(tris, np.float64).reshape(-1, 3, 3)[:, 0]),
        axis=-1))[None, :] < 1e-12)
    return np.any(edge | interval | (degenerate & inside), axis=1)


def occluded64(tris: np.ndarray, rays: np.ndarray) -> np.ndarray:
    t, u, v, ok = solve_tuv(tris, rays)
    ry = np.asarray(rays, np.float64).reshape(-1, 8)
    inside = ok & (u >= 0) & (v >= 0) & (u + v <= 1) & (t > ry[:, 3:4]) & (t < ry[:, 7:8])
    return np.any(inside, axis=1)


def closest64(tris: np.ndarray, rays: np.ndarray):
    """fp64 closest (t, u, v, prim) with prim ties to the smaller id."""
    t, u, v, ok = solve_tuv(tris, rays)
    ry = np.asarray(rays, np.float64).reshape(-1, 8)
    inside = ok & (u >= 0) & (v >= 0) & (u + v <= 1) & (t > ry[:, 3:4]) & (t < ry[:, 7:8])
    tt = np.where(inside, t, np.inf)
    prim = np.argmin(tt, axis=1)
    rows = np.arange(tt.shape[0])
    best_t = tt[rows, prim]
    hit = np.isfinite(best_t)
    return best_t, u[rows, prim], v[rows, prim], np.where(hit, prim, 0xFFFFFFFF).astype(np.uint64)
