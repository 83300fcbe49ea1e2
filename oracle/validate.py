"""Structural validator for canonical BVHs (test infrastructure only).

Checks, independently of any builder: the node arrays form a depth-first
pre-order binary tree (left child = next node); every triangle appears in
exactly one leaf, leaves cover contiguous ranges in DFS order; leaf sizes are
within ``leaf_max``; each leaf box is the exact binary32 min/max of its
triangles' vertices and each interior box is the exact union of its
children's boxes; ``depth`` counts interior ancestors and stays within
``max_depth``.
"""
from __future__ import annotations

import numpy as np

NONE32 = 0xFFFFFFFF


def validate_bvh(bvh, tris: np.ndarray, leaf_max: int, max_depth: int) -> None:
    tris = np.asarray(tris, np.float32).reshape(-1, 3, 3)
    n = tris.shape[0]
    m = bvh.num_nodes
    if m != 2 * int(np.count_nonzero(bvh.right == NONE32)) - 1:
        raise AssertionError("node count is not 2*leaves-1")
    if not np.array_equal(np.sort(bvh.perm), np.arange(n, dtype=np.uint32)):
        raise AssertionError("triangle permutation is not a permutation")
    # walk the tree explicitly (iterative DFS) and check pre-order numbering
    expect_next = 0
    next_tri = 0
    stack = [(0, 0)]
    parent_of = np.full(m, -1, np.int64)
    while stack:
        node, depth = stack.pop()
        if node != expect_next:
            raise AssertionError(f"node {node} is not in DFS pre-order (expected {expect_next})")
        expect_next += 1
        if int(bvh.depth[node]) != depth:
            raise AssertionError(f"depth of node {node} is {bvh.depth[node]}, expected {depth}")
        if depth > max_depth:
            raise AssertionError("depth above max_depth")
        if bvh.right[node] == NONE32:
            c = int(bvh.count[node])
            if not (1 <= c <= leaf_max):
                raise AssertionError(f"leaf {node} has {c} triangles")
            if int(bvh.first[node]) != next_tri:
                raise AssertionError("leaves do not cover consecutive triangle ranges in DFS order")
            next_tri += c
        else:
            r = int(bvh.right[node])
            if not (node + 1 < r < m):
                raise AssertionError(f"bad right child {r} of node {node}")
            parent_of[node + 1] = node
            parent_of[r] = node
            stack.append((r, depth + 1))
            stack.append((node + 1, depth + 1))
    if expect_next != m or next_tri != n:
        raise AssertionError("tree does not cover all nodes / triangles")
    # boxes
    vt = tris[bvh.perm]                                   # BVH-ordered triangles
    tmin, tmax = vt.min(axis=1), vt.max(axis=1)           # exact binary32 min/max
    leaves = np.nonzero(bvh.right == NONE32)[0]
    for node in leaves:
        f, c = int(bvh.first[node]), int(bvh.count[node])
        want = np.concatenate([tmin[f:f + c].min(0), tmax[f:f + c].max(0)])
        if not np.array_equal(bvh.box[node], want):
            raise AssertionError(f"leaf {node} box is not the exact bound of its triangles")
    inner = np.nonzero(bvh.right != NONE32)[0]
    L, R = inner + 1, bvh.right[inner].astype(np.int64)
    want = np.concatenate([np.minimum(bvh.box[L, :3], bvh.box[R, :3]),
                           np.maximum(bvh.box[L, 3:], bvh.box[R, 3:])], axis=1)
    if not np.array_equal(bvh.box[inner], want):
        raise AssertionError("an interior box is not the exact union of its children")
