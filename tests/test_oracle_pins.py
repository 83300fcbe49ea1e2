"""Pins of the CPU oracle against things other than itself.

Each test ties an oracle function to the paper's rules, to mathematics
(fp64 linear algebra, exact rationals, the golden ratio), to brute force, or
to hand-computed values, so that a plausible slip in the oracle (a dropped
term, a wrong sign or index, a swapped operand) fails one of them.
"""
from __future__ import annotations

import os
from decimal import Decimal, getcontext
from fractions import Fraction

import itertools

import numpy as np
import pytest

import oracle
import scenegen as sg
from tests import fp64ref

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
NONE32 = 0xFFFFFFFF
EMPTY_TAG = np.uint64(0xFFFFFFFFFFFFFFFF)


def _ray(o, d, tmin=0.0, tmax=np.inf):
    return np.array([*o, tmin, *d, tmax], np.float32)


# ---------------------------------------------------------------------------
# Hash (grid origin + octahedral direction + Fibonacci fold)
# ---------------------------------------------------------------------------

def _golden_hash_cases():
    rows = []
    with open(os.path.join(GOLDEN, "hash_cases.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append([float(x) for x in line.split()])
    return rows


def _fields(key, qo, qd):
    key = int(key)
    m_o, m_d = (1 << qo) - 1, (1 << qd) - 1
    return (key & m_o, (key >> qo) & m_o, (key >> 2 * qo) & m_o,
            (key >> 3 * qo) & m_d, (key >> (3 * qo + qd)) & m_d)


def test_hash_hand_cases():
    cases = _golden_hash_cases()
    assert len(cases) >= 10
    for row in cases:
        qo, qd = int(row[0]), int(row[1])
        box = np.array(row[2:8], np.float32)
        ray = _ray(row[8:11], row[11:14])
        want = tuple(int(x) for x in row[14:19])
        keys, _ = oracle.hash_rays(box, qo, qd, 12, ray)
        assert _fields(keys[0], qo, qd) == want, (row, _fields(keys[0], qo, qd))
        assert int(keys[0]) >> (3 * qo + 2 * qd) == 0   # key has exactly 3qo+2qd bits


def test_hash_origin_cells_match_exact_rationals():
    g = np.random.default_rng(5)
    box = np.array([-0.3, 0.1, -2.0, 1.7, 0.35, 3.0], np.float32)
    qo = 5
    o = g.uniform(box[:3], box[3:], (2000, 3)).astype(np.float32)
    rays = np.concatenate([o, np.zeros((2000, 1)), np.tile([[0, 0, 1]], (2000, 1)), np.ones((2000, 1))], 1)
    keys, _ = oracle.hash_rays(box, qo, 4, 12, rays)
    checked = 0
    for i in range(2000):
        got = _fields(keys[i], qo, 4)[:3]
        for a in range(3):
            lo, hi = Fraction(float(box[a])), Fraction(float(box[3 + a]))
            x = (Fraction(float(o[i, a])) - lo) * (1 << qo) / (hi - lo)
            if abs(x - round(x)) < Fraction(1, 10 ** 4):
                continue          # binary32 rounding may legitimately fall either side
            checked += 1
            assert got[a] == min(max(int(x // 1), 0), (1 << qo) - 1)
    assert checked > 5000


def _octa_decode(u, v):
    """Inverse octahedral map (independent formulation): square -> unit vector."""
    z = 1.0 - abs(u) - abs(v)
    if z < 0:
        u, v = (1.0 - abs(v)) * (1 if u >= 0 else -1), (1.0 - abs(u)) * (1 if v >= 0 else -1)
    d = np.array([u, v, z])
    return d / np.linalg.norm(d)


def test_hash_octahedral_bins_contain_direction():
    g = np.random.default_rng(6)
    qd = 6
    d = g.normal(size=(3000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rays = np.concatenate([np.zeros((3000, 3)), np.zeros((3000, 1)), d, np.ones((3000, 1))], 1)
    keys, _ = oracle.hash_rays(np.array([0, 0, 0, 1, 1, 1], np.float32), 3, qd, 12, rays)
    cell = 2.0 / (1 << qd)
    for i in range(3000):
        bu, bv = _fields(keys[i], 3, qd)[3:]
        # the direction must decode into the bin: find the decoded position of
        # the direction on the square and check it lies in [b*cell-1, (b+1)*cell-1]
        # by testing that some point of the bin decodes to within the bin's
        # angular size (corners decode within ~ 2 cells of arc)
        cu, cv = (bu + 0.5) * cell - 1.0, (bv + 0.5) * cell - 1.0
        c = _octa_decode(cu, cv)
        ang = np.arccos(np.clip(np.dot(c, d[i]), -1, 1))
        assert ang < 2.5 * cell, (d[i], bu, bv, ang)


def test_hash_fibonacci_fold_matches_golden_ratio():
    # Knuth's multiplicative hashing: idx = floor(2^T * frac(key * (sqrt(5)-1)/2)),
    # with the 64-bit constant floor(2^64 / phi) standing in for 1/phi.
    getcontext().prec = 80
    inv_phi = (Decimal(5).sqrt() - 1) / 2
    g = np.random.default_rng(7)
    qo, qd, T = 5, 6, 20
    box = np.array([0, 0, 0, 1, 1, 1], np.float32)
    o = g.random((500, 3)).astype(np.float32)
    d = g.normal(size=(500, 3)).astype(np.float32)
    rays = np.concatenate([o, np.zeros((500, 1)), d, np.ones((500, 1))], 1)
    keys, idx = oracle.hash_rays(box, qo, qd, T, rays)
    checked = 0
    for k, i in zip(keys, idx):
        x = (Decimal(int(k)) * inv_phi) % 1 * (1 << T)
        if abs(x - x.to_integral_value()) < Decimal("1e-6"):
            continue
        checked += 1
        assert int(i) == int(x), (k, i, x)
    assert checked > 490
    # key 1 gives the leading T bits of 1/phi
    _, i1 = oracle.hash_rays(np.array([0, 0, 0, 1, 1, 1], np.float32), 5, 6, 12,
                             _ray([1 / 32 + 1e-3, 0, 0], [-1e-3, -1e-3, -1]))
    k1, _ = oracle.hash_rays(np.array([0, 0, 0, 1, 1, 1], np.float32), 5, 6, 12,
                             _ray([1 / 32 + 1e-3, 0, 0], [-1e-3, -1e-3, -1]))
    assert int(k1[0]) == 1
    assert _fields(1, 5, 6)[0] == 1 and int(i1[0]) == int(Decimal(4096) * inv_phi)


# ---------------------------------------------------------------------------
# Moller-Trumbore and slab test
# ---------------------------------------------------------------------------

def test_mt_matches_fp64_linear_solve():
    g = np.random.default_rng(8)
    tris = g.uniform(-1, 1, (400, 3, 3)).astype(np.float32)
    rays = np.concatenate([g.uniform(-2, 2, (400, 3)), np.zeros((400, 1)),
                           g.normal(size=(400, 3)), np.full((400, 1), np.inf)], 1).astype(np.float32)
    # aim half of the rays at the triangle to get hits
    tgt = tris.mean(axis=1) + g.uniform(-0.3, 0.3, (400, 3))
    rays[::2, 4:7] = (tgt[::2] - rays[::2, 0:3]).astype(np.float32)
    hits = mism = 0
    for k in range(400):
        t, u, v, ok = fp64ref.solve_tuv(tris[k:k + 1], rays[k:k + 1])
        t, u, v = float(t[0, 0]), float(u[0, 0]), float(v[0, 0])
        m = min(u, v, 1 - u - v)
        h, t32, u32, v32 = oracle.mt(tris[k], rays[k])
        if abs(m) < 1e-5:
            continue
        inside = m > 0
        assert h == inside, (k, m)
        if inside:
            hits += 1
            assert abs(t32 - t) <= 1e-5 * max(1.0, abs(t))
            assert abs(u32 - u) <= 1e-5 and abs(v32 - v) <= 1e-5
    assert hits > 60


def test_mt_hand_cases():
    tri = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32)
    # straight down onto (0.25, 0.25): t = 2, u = v = 0.25
    assert oracle.mt(tri, _ray([0.25, 0.25, 2], [0, 0, -1])) == (True, 2.0, 0.25, 0.25)
    # from below also hits (two-sided), t = 1
    assert oracle.mt(tri, _ray([0.25, 0.5, -1], [0, 0, 1])) == (True, 1.0, 0.25, 0.5)
    # parallel to the plane: det == 0 -> miss
    assert oracle.mt(tri, _ray([0.25, 0.25, 0], [1, 0, 0]))[0] is False
    # outside the hypotenuse u + v > 1
    assert oracle.mt(tri, _ray([0.6, 0.6, 1], [0, 0, -1]))[0] is False
    # exactly on the v = 0 edge counts as inside (closed triangle)
    assert oracle.mt(tri, _ray([0.5, 0.0, 1], [0, 0, -1]))[0] is True
    # behind the origin still reports t < 0 (the caller applies the interval)
    h, t, _, _ = oracle.mt(tri, _ray([0.25, 0.25, -3], [0, 0, -1]))
    assert h and t == -3.0


def test_slab_cases():
    box = np.array([0, 0, 0, 1, 1, 1], np.float32)
    assert oracle.slab(box, _ray([-1, 0.5, 0.5], [1, 0, 0]), np.inf) == (True, 1.0)
    assert oracle.slab(box, _ray([-1, 0.5, 0.5], [1, 0, 0]), 0.99)[0] is False      # interval ends before
    assert oracle.slab(box, _ray([-1, 0.5, 0.5], [-1, 0, 0]), np.inf)[0] is False   # pointing away
    assert oracle.slab(box, _ray([-1, 2.0, 0.5], [1, 0, 0]), np.inf)[0] is False    # passes above
    # origin inside: tnear clamps to tmin
    assert oracle.slab(box, _ray([0.5, 0.5, 0.5], [0, 1, 0], tmin=0.25), np.inf) == (True, 0.25)
    # ray lying in the plane x = 0 of a face, d.x = 0: (0 - 0) * inf is NaN and
    # is ignored, the far face gives +inf, so the slab is empty (a miss)
    assert oracle.slab(box, _ray([0, 0.5, -1], [0, 0, 1]), np.inf)[0] is False
    # same ray against a box of zero thickness in x: both slab distances are NaN,
    # both are ignored, and the other axes decide (a hit)
    assert oracle.slab(np.array([0, 0, 0, 0, 1, 1], np.float32), _ray([0, 0.5, -1], [0, 0, 1]), np.inf) == (True, 1.0)
    # zero-thickness box (a flat leaf) is still hit
    flat = np.array([0, 0.5, 0, 1, 0.5, 1], np.float32)
    assert oracle.slab(flat, _ray([0.5, 2, 0.5], [0, -1, 0]), np.inf) == (True, 1.5)
    # grazing the edge x = 0, y = 1 diagonally: tnear == tfar exactly is a hit
    assert oracle.slab(box, _ray([-1, 0, 0.5], [1, 1, 0]), np.inf) == (True, 1.0)
    # lying in the top face plane y = 1 with d.y = 0 is outside (see above)
    assert oracle.slab(box, _ray([-1, 1, 0.5], [1, 0, 0]), np.inf)[0] is False


def test_slab_matches_fp64_intervals():
    g = np.random.default_rng(9)
    n_ok = 0
    for _ in range(3000):
        lo = g.uniform(-1, 1, 3)
        hi = lo + g.uniform(0, 1, 3)
        box = np.concatenate([lo, hi]).astype(np.float32)
        r = _ray(g.uniform(-3, 3, 3), g.normal(size=3))
        tcur = float(g.uniform(0.1, 10))
        o, d = r[0:3].astype(np.float64), r[4:7].astype(np.float64)
        b = box.astype(np.float64)
        t0, t1 = (b[:3] - o) / d, (b[3:] - o) / d
        tn = max(np.minimum(t0, t1).max(), 0.0)
        tf = min(np.maximum(t0, t1).min(), tcur)
        if abs(tn - tf) < 1e-5 * max(1, abs(tf)):
            continue
        n_ok += 1
        assert oracle.slab(box, r, tcur)[0] == (tn <= tf)
    assert n_ok > 2900


# ---------------------------------------------------------------------------
# BVH construction
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 3, 4, 5, 17, 256, 3000])
def test_sah_bvh_is_valid(n):
    tris = sg.triangle_soup(11 + n, n)
    b = oracle.build_sah(tris, leaf_max=4)
    oracle.validate_bvh(b, tris, 4, 64)


def test_bvh_degenerate_inputs():
    one = sg.triangle_soup(3, 1)
    same = np.repeat(one, 50, axis=0)                 # all centroids coincide -> halving splits
    b = oracle.build_sah(same, leaf_max=4)
    oracle.validate_bvh(b, same, 4, 64)
    assert b.max_depth() <= 5
    # depth cap is enforced
    with pytest.raises(ValueError):
        oracle.build_sah(same, leaf_max=1, max_depth=3)


def test_validator_catches_planted_mistakes():
    tris = sg.triangle_soup(4, 64)
    b = oracle.build_sah(tris)
    oracle.validate_bvh(b, tris, 4, 64)
    bad = oracle.CanonBVH(b.box.copy(), b.right, b.first, b.count, b.depth, b.perm)
    inner = np.nonzero(b.right != NONE32)[0][1]
    bad.box[inner, 4] = np.nextafter(bad.box[inner, 4], np.float32(2))   # one ulp too large
    with pytest.raises(AssertionError):
        oracle.validate_bvh(bad, tris, 4, 64)
    bad2 = oracle.CanonBVH(b.box, b.right, b.first, b.count, b.depth, b.perm.copy())
    bad2.perm[[0, -1]] = bad2.perm[[-1, 0]]   # two triangles trade leaves
    with pytest.raises(AssertionError):
        oracle.validate_bvh(bad2, tris, 4, 64)


def test_sah_beats_median_on_cost():
    # the SAH tree should need fewer box tests than median splits on a clustered scene
    tris = sg.triangle_soup(21, 2000)
    tris[:1000] *= 0.1
    rays = sg.tiny_shadow_rays(21, 2000)
    _, s_sah = oracle.trace(oracle.build_sah(tris), tris, rays)
    _, s_med = oracle.trace(oracle.build_median(tris), tris, rays)
    assert s_sah["box_tests"] < s_med["box_tests"]


def _point_tris(pts):
    """Degenerate triangles with all three vertices at each point."""
    pts = np.asarray(pts, np.float32).reshape(-1, 3)
    return np.ascontiguousarray(np.tile(pts, (1, 3)))


def test_lbvh_codes_hand_cases():
    # centres span [0, 2^21] on every axis, so a cell is the integer part of the
    # centre; cell (1, 2, 4) interleaves to bits 2 (x bit 0), 4 (y bit 1) and
    # 6 (z bit 2); the far corner clamps to 2^21 - 1 on every axis
    S = 2.0 ** 21
    tris = _point_tris([[0, 0, 0], [S, S, S], [1, 2, 4], [2 ** 20, 0, 0], [0, 2 ** 20 + 0.5, 0], [0, 0, 3]])
    c = oracle.lbvh_codes(tris).astype(object)
    assert c.tolist() == [0, 2 ** 63 - 1, 4 + 16 + 64, 2 ** 62, 2 ** 61, 1 + 8]
    # a flat axis has a single cell: every z bit stays 0
    flat = _point_tris([[0, 0, 5], [S, S, 5], [1, 1, 5]])
    assert oracle.lbvh_codes(flat).tolist() == [0, 0b110 * (2 ** 63 - 1) // 7, 0b110]
    # cells are cubes sized by the largest extent: with y spanning a quarter of
    # x, y's top cell is 2^19 (bit 19 -> code bit 58) and 2^18 lands on bit 55,
    # where per-axis cells would put them on bits 61 and 58
    flat_y = _point_tris([[0, 0, 0], [S, S / 4, 0], [S / 2, S / 8, 0]])
    x_all = sum(1 << (3 * k + 2) for k in range(21))
    assert oracle.lbvh_codes(flat_y).astype(object).tolist() == [0, x_all + 2 ** 58, 2 ** 62 + 2 ** 55]


def test_lbvh_equal_codes_split_by_position():
    # five copies of one triangle share a code, so the splits follow the
    # sorted positions' bits: [0,5) -> [0,4) + [4]; [0,4) -> [0,2) + [2,4)
    tris = np.repeat(sg.triangle_soup(5, 1), 5, axis=0)
    b = oracle.build_lbvh(tris, leaf_max=1)
    assert b.right.tolist() == [8, 5, 4, NONE32, NONE32, 7, NONE32, NONE32, NONE32]
    assert b.first[b.right == NONE32].tolist() == [0, 1, 2, 3, 4]
    assert b.depth.tolist() == [0, 1, 2, 3, 3, 2, 3, 3, 1]
    assert b.perm.tolist() == [0, 1, 2, 3, 4]          # equal codes keep primitive order
    with pytest.raises(ValueError):
        oracle.build_lbvh(np.repeat(tris, 10, axis=0), leaf_max=1, max_depth=3)


def _lbvh_keys(tris, b):
    code = oracle.lbvh_codes(tris)
    return [(int(code[p]) << 28) | k for k, p in enumerate(b.perm.tolist())], code


@pytest.mark.parametrize("n,leaf_max", [(1, 4), (4, 4), (5, 4), (97, 1), (700, 2), (3000, 4)])
def test_lbvh_is_the_radix_tree_of_the_sorted_codes(n, leaf_max):
    # independent of the builder: the tree is valid, its triangles are in
    # (code, id) order, a node is a leaf exactly when it holds <= leaf_max
    # triangles, and each split leaves both children a longer common prefix of
    # the key (code, position) than their parent; for sorted distinct keys
    # only the radix-tree split does that
    tris = sg.triangle_soup(40 + n, n)
    if n >= 700:
        tris[: n // 3] = tris[n // 3: 2 * (n // 3)]        # many equal codes
    b = oracle.build_lbvh(tris, leaf_max=leaf_max)
    oracle.validate_bvh(b, tris, leaf_max, 64)
    keys, code = _lbvh_keys(tris, b)
    order = sorted(range(n), key=lambda t: (int(code[t]), t))
    assert b.perm.tolist() == order

    def prefix(lo, hi):        # common leading bits of keys[lo .. hi-1], 91-bit keys
        return 91 - (keys[lo] ^ keys[hi - 1]).bit_length()

    rng = {}
    for i in range(b.num_nodes - 1, -1, -1):
        if b.right[i] == NONE32:
            rng[i] = (int(b.first[i]), int(b.first[i] + b.count[i]))
            assert rng[i][1] - rng[i][0] <= leaf_max
        else:
            L, R = rng[i + 1], rng[int(b.right[i])]
            assert L[1] == R[0]
            rng[i] = (L[0], R[1])
            assert rng[i][1] - rng[i][0] > leaf_max
            p = prefix(*rng[i])
            for lo, hi in (L, R):
                assert hi - lo == 1 or prefix(lo, hi) > p


# ---------------------------------------------------------------------------
# Treelet restructuring of the linear BVH (Karras and Aila, HPG 2013)
# ---------------------------------------------------------------------------

def _all_trees(items):
    """Every full binary tree on the leaves `items`, children unordered, as
    nested pairs: (2k - 3)!! trees for k leaves."""
    if len(items) == 1:
        yield items[0]
        return
    first, rest = items[0], items[1:]
    for r in range(len(rest)):
        for comb in itertools.combinations(rest, r):
            other = [x for x in rest if x not in comb]
            for a in _all_trees([first, *comb]):
                for b in _all_trees(other):
                    yield (a, b)


def _tree_cost64(tree, lo, hi):
    """(box lo, box hi, sum of the half areas of the interior nodes), fp64."""
    if not isinstance(tree, tuple):
        return lo[tree], hi[tree], 0.0
    la, ha, ca = _tree_cost64(tree[0], lo, hi)
    lb, hb, cb = _tree_cost64(tree[1], lo, hi)
    l, h = np.minimum(la, lb), np.maximum(ha, hb)
    d = h - l
    return l, h, ca + cb + float(d[0] * d[1] + d[1] * d[2] + d[2] * d[0])


def _bvh_cost64(b):
    inner = b.right != NONE32
    d = b.box[inner, 3:].astype(np.float64) - b.box[inner, :3].astype(np.float64)
    return float((d[:, 0] * d[:, 1] + d[:, 1] * d[:, 2] + d[:, 2] * d[:, 0]).sum())


def test_treelet_count_of_trees():
    assert [sum(1 for _ in _all_trees(list(range(k)))) for k in range(1, 8)] == [1, 1, 3, 15, 105, 945, 10395]


@pytest.mark.parametrize("k", [3, 4, 5, 6, 7])
def test_treelet_pass_finds_the_optimal_tree_of_seven_leaves(k):
    # with at most 7 leaves the root's treelet holds every leaf, so one pass
    # must reach the least sum of interior half areas over all (2k-3)!! trees
    worse = 0
    for seed in range(12):
        tris = sg.triangle_soup(900 + 17 * k + seed, k, edge=0.3)
        v = tris.reshape(-1, 3, 3).astype(np.float64)
        lo, hi = v.min(1), v.max(1)
        best = min(_tree_cost64(t, lo, hi)[2] for t in _all_trees(list(range(k))))
        b = oracle.build_lbvh(tris, leaf_max=1, treelet_passes=1)
        oracle.validate_bvh(b, tris, 1, 64)
        assert _bvh_cost64(b) == pytest.approx(best, rel=1e-6), seed
        worse += _bvh_cost64(oracle.build_lbvh(tris, leaf_max=1)) > best * (1 + 1e-6)
    assert worse >= 3          # the radix tree alone is often not optimal


@pytest.mark.parametrize("n,leaf_max", [(50, 1), (1000, 2), (5000, 4)])
def test_treelet_passes_keep_leaves_and_lower_the_cost(n, leaf_max):
    tris = sg.triangle_soup(300 + n, n)
    base = oracle.build_lbvh(tris, leaf_max=leaf_max)

    def leaf_sets(b):
        lf = np.nonzero(b.right == NONE32)[0]
        return sorted(tuple(sorted(b.perm[b.first[i]:b.first[i] + b.count[i]].tolist())) for i in lf)

    prev = _bvh_cost64(base)
    for p in (1, 2, 3):
        b = oracle.build_lbvh(tris, leaf_max=leaf_max, treelet_passes=p)
        oracle.validate_bvh(b, tris, leaf_max, 64)
        assert leaf_sets(b) == leaf_sets(base)
        c = _bvh_cost64(b)
        assert c <= prev * (1 + 1e-6)
        prev = c
    assert prev < _bvh_cost64(base) * 0.99
    assert oracle.build_lbvh(tris, leaf_max=leaf_max, treelet_passes=0).perm.tolist() == base.perm.tolist()


# ---------------------------------------------------------------------------
# Traversal versus brute force (plain definitions of any-hit and closest hit)
# ---------------------------------------------------------------------------

def _allowed_mismatch(tris, rays, bad):
    if not np.any(bad):
        return
    idx = np.nonzero(bad)[0]
    ne = fp64ref.near_edge(tris, rays[idx])
    assert np.all(ne), f"{int((~ne).sum())} mismatches away from any triangle edge: rays {idx[~ne][:10]}"


def _tiny_scene_rays(seed):
    g = np.random.default_rng(seed)
    n = int(g.integers(1, 200))
    tris = sg.triangle_soup(seed, n, edge=float(g.uniform(0.05, 0.4)))
    m = 300
    o = g.uniform(-0.2, 1.2, (m, 3))
    tgt = g.uniform(0, 1, (m, 3))
    d = tgt - o
    tmax = np.where(g.random(m) < 0.5, 1.0, np.inf)
    rays = sg.pack_rays(o.astype(np.float32), d.astype(np.float32), 0.0, tmax)
    return tris, rays


def test_config1_anyhit_matches_bruteforce():
    tris = sg.triangle_soup(1, 256)
    rays = sg.tiny_shadow_rays(1, 4096)
    b = oracle.build_sah(tris)
    occ, st = oracle.trace(b, tris, rays)
    bf = oracle.brute_force(tris, rays)
    _allowed_mismatch(tris, rays, occ != bf)
    assert st["hits"] == int(occ.sum()) and st["rays"] == 4096
    # fp64 agrees except near edges
    o64 = fp64ref.occluded64(tris, rays)
    _allowed_mismatch(tris, rays, o64 != occ.astype(bool))


@pytest.mark.parametrize("seed", range(30))
def test_random_tiny_scenes_match_bruteforce(seed):
    tris, rays = _tiny_scene_rays(100 + seed)
    b = oracle.build_sah(tris)
    occ, _ = oracle.trace(b, tris, rays)
    _allowed_mismatch(tris, rays, occ != oracle.brute_force(tris, rays))
    hits, _ = oracle.trace(b, tris, rays, query="closest", mode="exact")
    bfh = oracle.brute_force(tris, rays, closest=True)
    _allowed_mismatch(tris, rays, np.any(hits.view(np.uint32) != bfh.view(np.uint32), axis=1))
    # fp64 closest: t within 1e-5 relative, barycentrics within 1e-5
    t64, u64, v64, p64 = fp64ref.closest64(tris, rays)
    prim = hits[:, 3].view(np.uint32).astype(np.uint64)
    same = prim == p64
    ne = fp64ref.near_edge(tris, rays)
    assert np.all(same | ne)
    h = same & (p64 != 0xFFFFFFFF)
    # binary32 Moller-Trumbore error grows as the ray grazes the plane: hold the
    # 1e-5 bound where the ray meets the plane at more than ~6 degrees
    tri = tris.astype(np.float64)[p64[h].astype(np.int64)]
    nrm = np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0])
    d = rays[h, 4:7].astype(np.float64)
    cos = np.abs(np.sum(nrm * d, 1)) / (np.linalg.norm(nrm, axis=1) * np.linalg.norm(d, axis=1))
    tol = np.where(cos > 0.1, 1e-5, 1e-3)
    assert np.all(np.abs(hits[h, 0] - t64[h]) <= tol * np.maximum(1, np.abs(t64[h])))
    assert np.all(np.abs(hits[h, 1] - u64[h]) <= tol) and np.all(np.abs(hits[h, 2] - v64[h]) <= tol)


def test_results_do_not_depend_on_tree_shape():
    tris = sg.triangle_soup(31, 500)
    rays = sg.tiny_shadow_rays(31, 3000)
    a = oracle.build_sah(tris)
    m = oracle.build_median(tris)
    oa, _ = oracle.trace(a, tris, rays)
    om, _ = oracle.trace(m, tris, rays)
    _allowed_mismatch(tris, rays, oa != om)
    ha, _ = oracle.trace(a, tris, rays, query="closest", mode="exact")
    hm, _ = oracle.trace(m, tris, rays, query="closest", mode="exact")
    _allowed_mismatch(tris, rays, np.any(ha.view(np.uint32) != hm.view(np.uint32), axis=1))
    for lb in (oracle.build_lbvh(tris), oracle.build_lbvh(tris, treelet_passes=2)):
        ol, _ = oracle.trace(lb, tris, rays)
        _allowed_mismatch(tris, rays, oa != ol)
        hl, _ = oracle.trace(lb, tris, rays, query="closest", mode="exact")
        _allowed_mismatch(tris, rays, np.any(ha.view(np.uint32) != hl.view(np.uint32), axis=1))


def test_invalid_rays_are_counted_misses():
    tris = sg.triangle_soup(1, 64)
    b = oracle.build_sah(tris)
    rays = np.stack([
        _ray([0.5, -1, 0.5], [0, 0, 0]),            # zero direction
        _ray([np.nan, 0, 0], [0, 1, 0]),            # NaN origin
        _ray([0.5, -1, 0.5], [0, np.inf, 0]),       # infinite direction
        _ray([0.5, -1, 0.5], [0, 1, 0], 1.0, 1.0),  # empty interval
        _ray([0.5, -1, 0.5], [0, 1, 0], np.nan, 5), # NaN tmin
    ])
    occ, st = oracle.trace(b, tris, rays, table=oracle.Table(8, 4, 5, 6), epoch=2)
    assert occ.tolist() == [0] * 5 and st["invalid"] == 5 and st["lookups"] == 0 and st["traversals"] == 0
    hits, st = oracle.trace(b, tris, rays, query="closest")
    assert np.all(np.isinf(hits[:, 0])) and np.all(hits[:, 3].view(np.uint32) == NONE32)


# ---------------------------------------------------------------------------
# Counters on hand-built trees
# ---------------------------------------------------------------------------

def _hand_bvh(tris, nodes):
    """nodes: list of (right, first, count, depth) in DFS order; boxes computed exactly."""
    m = len(nodes)
    box = np.zeros((m, 6), np.float32)
    right = np.array([n[0] for n in nodes], np.uint32)
    first = np.array([n[1] for n in nodes], np.uint32)
    count = np.array([n[2] for n in nodes], np.uint32)
    depth = np.array([n[3] for n in nodes], np.uint32)
    t = np.asarray(tris, np.float32).reshape(-1, 3, 3)

    def fill(i):
        if right[i] == NONE32:
            v = t[first[i]:first[i] + count[i]].reshape(-1, 3)
            box[i] = np.concatenate([v.min(0), v.max(0)])
        else:
            fill(i + 1)
            fill(int(right[i]))
            box[i] = np.concatenate([np.minimum(box[i + 1, :3], box[right[i], :3]),
                                     np.maximum(box[i + 1, 3:], box[right[i], 3:])])
    fill(0)
    return oracle.CanonBVH(box, right, first, count, depth, np.arange(t.shape[0], dtype=np.uint32))


def _square(x0, z0, y, s=1.0):
    return np.array([[[x0, y, z0], [x0 + s, y, z0], [x0 + s, y, z0 + s]],
                     [[x0, y, z0], [x0 + s, y, z0 + s], [x0, y, z0 + s]]], np.float32)


def test_counters_single_leaf():
    tris = _square(0, 0, 0)
    b = _hand_bvh(tris, [(NONE32, 0, 2, 0)])
    oracle.validate_bvh(b, tris, 4, 64)
    rays = np.stack([_ray([0.5, 1, 0.25], [0, -1, 0]), _ray([3, 1, 3], [0, -1, 0])])
    occ, st = oracle.trace(b, tris, rays)
    # ray 0: root box test, visit the leaf, first triangle (0.5,0.25) lies in
    # triangle 0 (below the diagonal z < x) -> 1 triangle test.
    # ray 1: misses the root box -> 1 box test, nothing else.
    assert occ.tolist() == [1, 0]
    assert (st["box_tests"], st["nodes_visited"], st["leaf_visited"], st["tri_tests"]) == (2, 1, 1, 1)
    assert st["interior_visited"] == 0 and st["traversals"] == 2


def test_counters_two_and_three_leaves():
    # leaf A: square at x in [0,1] y=0; leaf C: same square at y=-1 (below A);
    # leaf B: x in [2,3] y=0
    tris = np.concatenate([_square(0, 0, 0), _square(0, 0, -1), _square(2, 0, 0)])
    # tree: root(0) -> [inner(1) -> leaf A(2), leaf C(3)] , leaf B(4)
    b = _hand_bvh(tris, [(4, 0, 0, 0), (3, 0, 0, 1), (NONE32, 0, 2, 2), (NONE32, 2, 2, 2), (NONE32, 4, 2, 1)])
    oracle.validate_bvh(b, tris, 4, 64)
    down = _ray([0.75, 1, 0.25], [0, -1, 0])
    occ, st = oracle.trace(b, tris, down[None])
    # root test (1); root interior: test inner(1) and B(4) -> only inner hit (2);
    # inner: test A and C -> both hit, A nearer (t=1 < 2), push C (2);
    # leaf A: triangle 0 holds (0.75, 0.25) -> hit on the first test, stop.
    assert occ.tolist() == [1]
    assert (st["box_tests"], st["interior_visited"], st["leaf_visited"], st["tri_tests"], st["nodes_visited"]) == \
        (5, 2, 1, 1, 3)
    # closest hit: A first gives t=1; C is popped with tnear=2 > 1 -> discarded, not visited
    hits, st = oracle.trace(b, tris, down[None], query="closest", mode="exact")
    assert hits[0, 0] == 1.0 and hits[0, 3].view(np.uint32) == 0
    assert (st["box_tests"], st["leaf_visited"], st["tri_tests"], st["nodes_visited"]) == (5, 1, 2, 3)
    # a ray from below reaches C first, then A is popped (tnear 1 < hit t? no: t(C) = 1, A at t=2 -> discarded)
    up = _ray([0.75, -2, 0.25], [0, 1, 0])
    hits, st = oracle.trace(b, tris, up[None], query="closest", mode="exact")
    assert hits[0, 0] == 1.0 and hits[0, 3].view(np.uint32) == 2
    assert (st["box_tests"], st["leaf_visited"], st["tri_tests"], st["nodes_visited"]) == (5, 1, 2, 3)
    # any-hit from below with an interval that stops short of C: boxes hit? C at t=1 excluded
    short = _ray([0.75, -2, 0.25], [0, 1, 0], 0.0, 0.5)
    occ, st = oracle.trace(b, tris, short[None])
    assert occ.tolist() == [0] and st["box_tests"] == 1 and st["nodes_visited"] == 0


# ---------------------------------------------------------------------------
# Predictor: paper rules and invariants
# ---------------------------------------------------------------------------

def _check_table_invariants(tb: oracle.Table, valid_leaves: set):
    used = tb.tags != EMPTY_TAG
    s = tb.slots
    # tag present <=> slot 0 present
    assert np.array_equal(used, s[:, 0] != NONE32)
    for row in s[used]:
        vals = [int(x) for x in row if x != NONE32]
        k = len(vals)
        assert all(int(x) == NONE32 for x in row[k:]), "slots not dense from slot 0"
        assert len(set(vals)) == k, "duplicate leaf in one entry (paper: no duplicates)"
        assert set(vals) <= valid_leaves


def _config1(epoch, nthreads=0, table=None, query="any", mode="paper"):
    tris = sg.triangle_soup(1, 256)
    rays = sg.tiny_shadow_rays(1, 4096)
    b = oracle.build_sah(tris)
    tb = table if table is not None else oracle.Table(12, 4, 5, 6)
    out = np.zeros(4096, np.uint8)
    res, st = oracle.trace(b, tris, rays, query=query, mode=mode, table=tb, epoch=epoch, nthreads=nthreads,
                           outcome=out)
    return tris, rays, b, tb, res, st, out


def test_prediction_hits_are_true_hits():
    tris, rays, b, tb, occ, st, out = _config1(256)
    bf = oracle.brute_force(tris, rays)
    assert st["pred_hits"] > 0
    assert np.all(bf[out == 2] == 1)                 # predicted-hit => true hit
    assert np.all(occ[out == 2] == 1)
    _allowed_mismatch(tris, rays, occ != bf)          # any-hit answers are unaffected
    assert st["positives"] == st["pred_hits"] + st["false_pos"]
    assert st["traversals"] + st["pred_hits"] == st["lookups"] == 4096 - st["invalid"]
    _check_table_invariants(tb, set(int(x) for x in b.leaf_ids()))


@pytest.mark.parametrize("epoch", [1, 256, 4096])
def test_table_invariants_and_counter_identities(epoch):
    tris, rays, b, tb, occ, st, out = _config1(epoch)
    _check_table_invariants(tb, set(int(x) for x in b.leaf_ids()))
    assert st["records"] == st["hits"] - st["pred_hits"]
    assert st["leaf_inserts"] + st["dropped"] <= st["records"]
    used = int(np.count_nonzero(tb.tags != EMPTY_TAG))
    assert used <= st["tag_claims"]
    assert int(np.count_nonzero(tb.slots != NONE32)) <= st["leaf_inserts"]


def test_single_epoch_equals_plain():
    tris, rays, b, tb, occ, st, out = _config1(4096)
    occ_p, st_p = oracle.trace(b, tris, rays)
    assert np.array_equal(occ, occ_p)
    assert st["positives"] == 0 and st["pred_hits"] == 0
    for k in ("nodes_visited", "interior_visited", "leaf_visited", "box_tests", "tri_tests", "traversals", "hits"):
        assert st[k] == st_p[k], k
    assert st["records"] == st["hits"]


def test_null_predictor_equals_plain_everywhere():
    tris = sg.triangle_soup(1, 256)
    rays = sg.tiny_shadow_rays(1, 4096)
    b = oracle.build_sah(tris)
    h1, s1 = oracle.trace(b, tris, rays, query="closest", mode="paper")
    h2, s2 = oracle.trace(b, tris, rays, query="closest", mode="exact")
    assert np.array_equal(h1.view(np.uint32), h2.view(np.uint32)) and s1 == s2


def test_determinism_over_thread_counts():
    res = []
    for nt in (1, 3, 8):
        tris, rays, b, tb, occ, st, out = _config1(256, nthreads=nt)
        res.append((occ.tobytes(), tb.tags.tobytes(), tb.slots.tobytes(), tuple(sorted(st.items()))))
    assert res[0] == res[1] == res[2]


def test_paper_closest_invariants():
    tris = sg.triangle_soup(41, 300, edge=0.15)
    g = np.random.default_rng(41)
    o = np.tile([[0.5, -0.5, 0.5]], (3000, 1)) + g.uniform(-0.02, 0.02, (3000, 3))
    d = np.tile([[0.0, 1.0, 0.0]], (3000, 1)) + g.uniform(-0.25, 0.25, (3000, 3))
    rays = sg.pack_rays(o.astype(np.float32), d.astype(np.float32), 0.0, np.inf)
    b = oracle.build_sah(tris)
    tb = oracle.Table(14, 8, 5, 6)
    out = np.zeros(3000, np.uint8)
    hp, st = oracle.trace(b, tris, rays, query="closest", mode="paper", table=tb, epoch=64, outcome=out)
    he, _ = oracle.trace(b, tris, rays, query="closest", mode="exact")
    assert st["pred_hits"] > 100
    prim = hp[:, 3].view(np.uint32)
    hit = prim != NONE32
    # the returned triangle really intersects at the returned t
    for i in np.nonzero(hit)[0]:
        h, t, u, v = oracle.mt(tris[prim[i]], rays[i])
        assert h and t == hp[i, 0] and u == hp[i, 1] and v == hp[i, 2]
    # never closer than the exact closest hit, and never a miss when one exists
    assert np.all(hp[hit, 0] >= he[hit, 0])
    assert np.array_equal(hit, he[:, 3].view(np.uint32) != NONE32)
    # rays that did not succeed by prediction equal the exact answer bit for bit
    trav = out != 2
    assert np.array_equal(hp[trav].view(np.uint32), he[trav].view(np.uint32))
    # and some predictions are (legitimately, per the paper) not the closest
    assert np.any(hp[:, 0] > he[:, 0]) or st["pred_hits"] > 0


def test_exact_closest_with_predictor_is_exact():
    tris = sg.triangle_soup(42, 300, edge=0.15)
    g = np.random.default_rng(42)
    o = np.tile([[0.5, -0.5, 0.5]], (2000, 1)) + g.uniform(-0.02, 0.02, (2000, 3))
    d = np.tile([[0.0, 1.0, 0.0]], (2000, 1)) + g.uniform(-0.25, 0.25, (2000, 3))
    rays = sg.pack_rays(o.astype(np.float32), d.astype(np.float32), 0.0, np.inf)
    b = oracle.build_sah(tris)
    tb = oracle.Table(14, 8, 5, 6)
    hx, st = oracle.trace(b, tris, rays, query="closest", mode="exact", table=tb, epoch=64)
    he, st0 = oracle.trace(b, tris, rays, query="closest", mode="exact")
    assert np.array_equal(hx.view(np.uint32), he.view(np.uint32))
    assert st["pred_hits"] > 0 and st["nodes_skipped"] == 0
    # the predicted bound can only shrink the traversal
    assert st["interior_visited"] <= st0["interior_visited"]


def _sequential_model(tris, rays, bvh, qo, qd):
    """The paper's sequential predictor (an unbounded dict, no replacement):
    a hit-all ray looks up its hash; if present, the stored leaves are
    tested (each leaf's box first, against the best hit so far) and the best
    hit there is accepted; otherwise (or on a miss there) the ray traverses
    and its result leaf is appended if absent."""
    keys, _ = oracle.hash_rays(bvh.box[0], qo, qd, 31, rays)
    leaf_of_pos = {}
    box_of_leaf = {}
    for i in np.nonzero(bvh.right == NONE32)[0]:
        lid = (int(bvh.first[i]) << 3) | (int(bvh.count[i]) - 1)
        box_of_leaf[lid] = bvh.box[i]
        for k in range(int(bvh.first[i]), int(bvh.first[i] + bvh.count[i])):
            leaf_of_pos[k] = lid
    pos_of_prim = {int(p): k for k, p in enumerate(bvh.perm)}
    exact = oracle.brute_force(tris, rays, closest=True)
    table, out, pred_hits = {}, [], 0
    for i in range(rays.shape[0]):
        k = int(keys[i])
        best = None
        for lid in table.get(k, []):
            if not oracle.slab(box_of_leaf[lid], rays[i], best[0] if best is not None else float(rays[i, 7]))[0]:
                continue
            f, c = lid >> 3, (lid & 7) + 1
            for pos in range(f, f + c):
                prim = int(bvh.perm[pos])
                h, t, u, v = oracle.mt(tris[prim], rays[i])
                if h and rays[i, 3] < t < rays[i, 7] and (best is None or (t, prim) < best[:2]):
                    best = (t, prim)
        if best is not None:
            pred_hits += 1
            out.append(best[1])
            continue
        prim = int(exact[i, 3].view(np.uint32))
        out.append(prim)
        if prim != NONE32:
            lid = leaf_of_pos[pos_of_prim[prim]]
            lst = table.setdefault(k, [])
            if lid not in lst:
                lst.append(lid)
    return table, out, pred_hits


def test_epoch_one_equals_paper_sequential_semantics():
    tris = sg.triangle_soup(43, 200, edge=0.15)
    g = np.random.default_rng(43)
    o = np.tile([[0.5, -0.5, 0.5]], (600, 1)) + g.uniform(-0.05, 0.05, (600, 3))
    d = np.tile([[0.0, 1.0, 0.0]], (600, 1)) + g.uniform(-0.3, 0.3, (600, 3))
    rays = sg.pack_rays(o.astype(np.float32), d.astype(np.float32), 0.0, np.inf)
    b = oracle.build_sah(tris)
    qo, qd, T, W = 4, 4, 22, 8
    keys, idx = oracle.hash_rays(b.box[0], qo, qd, T, rays)
    # no two distinct keys share an index: the finite table behaves like a dict
    pairs = set(zip(idx.tolist(), keys.tolist()))
    assert len({i for i, _ in pairs}) == len(pairs)
    model, prims, pred_hits = _sequential_model(tris, rays, b, qo, qd)
    assert max(len(v) for v in model.values()) <= W
    tb = oracle.Table(T, W, qo, qd)
    hp, st = oracle.trace(b, tris, rays, query="closest", mode="paper", table=tb, epoch=1)
    assert st["pred_hits"] == pred_hits > 20
    assert hp[:, 3].view(np.uint32).tolist() == prims
    got = {}
    for i in np.nonzero(tb.tags != EMPTY_TAG)[0]:
        got[int(tb.tags[i])] = [int(x) for x in tb.slots[i] if x != NONE32]
    assert got == model


def _three_squares():
    # three 0.3 x 0.3 squares on y = 0, far enough apart to sit in separate leaves
    tris = np.concatenate([_square(0.0, 0.0, 0.0, 0.3), _square(0.35, 0.0, 0.0, 0.3), _square(0.7, 0.0, 0.0, 0.3)])
    b = oracle.build_sah(tris, leaf_max=2)
    leaf_of_prim = {}
    for i in np.nonzero(b.right == NONE32)[0]:
        for k in range(int(b.first[i]), int(b.first[i] + b.count[i])):
            leaf_of_prim[int(b.perm[k])] = (int(b.first[i]) << 3) | (int(b.count[i]) - 1)
    sq_leaf = [leaf_of_prim[2 * q] for q in range(3)]
    assert all(leaf_of_prim[2 * q + 1] == sq_leaf[q] for q in range(3)) and len(set(sq_leaf)) == 3
    return tris, b, sq_leaf


def _rays_to_squares(origin, squares, seed):
    g = np.random.default_rng(seed)
    x0 = np.array([0.0, 0.35, 0.7])[squares]
    tgt = np.stack([x0 + g.uniform(0.05, 0.25, len(squares)), np.zeros(len(squares)),
                    g.uniform(0.05, 0.25, len(squares))], 1)
    o = np.tile(np.asarray(origin, np.float64), (len(squares), 1))
    return sg.pack_rays(o.astype(np.float32), (tgt - o).astype(np.float32), 0.0, 2.0)


def test_update_rule_capacity_hand_case():
    # qo = qd = 1: every ray from (-0.5, 1, 0.1) towards the squares has
    # cell (0, 0, 0) (x clamped, y axis flat -> scale 0, z = floor(0.667))
    # and direction bins (1, 0) (px > 0, py < 0, no fold): key = 1 << 3 = 8.
    tris, b, sq_leaf = _three_squares()
    squares = np.array([2, 0, 1] * 10)
    rays = _rays_to_squares([-0.5, 1.0, 0.1], squares, 50)
    keys, _ = oracle.hash_rays(b.box[0], 1, 1, 4, rays)
    assert set(keys.tolist()) == {8}
    for W in (1, 2):
        tb = oracle.Table(4, W, 1, 1)
        _, st = oracle.trace(b, tris, rays, query="closest", mode="exact", table=tb, epoch=30)
        entry = np.nonzero(tb.tags != EMPTY_TAG)[0]
        assert len(entry) == 1 and int(tb.tags[entry[0]]) == 8
        # leaves in the order of the first ray that reached each: squares 2, 0, 1
        kept = [sq_leaf[2], sq_leaf[0], sq_leaf[1]][:W]
        assert tb.slots[entry[0]].tolist() == kept
        assert (st["records"], st["tag_claims"], st["leaf_inserts"], st["conflicts"]) == (30, 1, W, 0)
        assert st["dropped"] == sum(1 for q in squares if sq_leaf[q] not in kept)
    # a later epoch keeps the entry (same key) and only appends into free slots
    tb = oracle.Table(4, 2, 1, 1)
    oracle.trace(b, tris, rays[squares == 0], query="closest", mode="exact", table=tb, epoch=1000)
    _, st = oracle.trace(b, tris, rays[squares != 0], query="closest", mode="exact", table=tb, epoch=1000)
    e = int(np.nonzero(tb.tags != EMPTY_TAG)[0][0])
    # the second call's first ray reaches square 2: its leaf takes the free slot
    assert tb.slots[e].tolist() == [sq_leaf[0], sq_leaf[2]]
    assert st["tag_claims"] == 0 and st["leaf_inserts"] == 1 and st["positives"] == 20


def _first_distinct(seq):
    return list(dict.fromkeys(seq))


@pytest.mark.parametrize("order", [(0, 1, 2), (2, 1, 0), (1, 2, 0), (2, 0, 2, 1), (1, 1, 0, 1, 2), (0, 2, 0, 1, 2)])
def test_update_rule_earliest_ray_wins_a_full_entry(order):
    # More distinct leaves than slots compete for one entry (one key, one
    # epoch).  The smallest ray id wins any conflict: leaves enter in the order
    # of the first ray that reached each, and the later ones are dropped.  A
    # rule that fills by leaf id (the squares' leaf ids increase with the
    # square) keeps 0, 1 whatever the order, and fails the orders that start
    # with square 2 or reach square 2 before square 1.
    tris, b, sq_leaf = _three_squares()
    assert sq_leaf == sorted(sq_leaf)
    squares = np.array(list(order) * 4)
    rays = _rays_to_squares([-0.5, 1.0, 0.1], squares, 70 + len(order))
    for W in (1, 2, 3):
        tb = oracle.Table(4, W, 1, 1)
        _, st = oracle.trace(b, tris, rays, query="closest", mode="exact", table=tb, epoch=len(squares))
        e = int(np.nonzero(tb.tags != EMPTY_TAG)[0][0])
        kept = [sq_leaf[q] for q in _first_distinct(order)][:W]
        assert [x for x in tb.slots[e].tolist() if x != NONE32] == kept, (order, W)
        assert st["leaf_inserts"] == len(kept)
        assert st["dropped"] == sum(1 for q in squares if sq_leaf[q] not in kept)
    # FIFO: the first W of them, in that order, as well
    tb = oracle.Table(4, 2, 1, 1, policy=1)
    oracle.trace(b, tris, rays, query="closest", mode="exact", table=tb, epoch=len(squares))
    e = int(np.nonzero(tb.tags != EMPTY_TAG)[0][0])
    assert tb.slots[e].tolist() == [sq_leaf[q] for q in _first_distinct(order)][:2]


def test_update_rule_smallest_ray_id_owns_the_entry():
    tris, b, sq_leaf = _three_squares()
    # rays from below, (-0.5, -1, 0.1) upwards: same cell, bins (1, 1) -> key 8 + 16 = 24.
    # In a 2-entry table keys 8 and 24 share index 1 (top bit of k * 0x9E3779B97F4A7C15).
    below = _rays_to_squares([-0.5, -1.0, 0.1], np.array([1] * 5), 53)
    above = _rays_to_squares([-0.5, 1.0, 0.1], np.array([0, 2] * 10), 54)
    for order, owner in ((np.concatenate([below, above]), 24), (np.concatenate([above, below]), 8)):
        keys, idx = oracle.hash_rays(b.box[0], 1, 1, 1, order)
        assert set(keys.tolist()) == {8, 24} and set(idx.tolist()) == {1}
        tb = oracle.Table(1, 4, 1, 1)
        _, st = oracle.trace(b, tris, order, query="closest", mode="exact", table=tb, epoch=100)
        assert int(tb.tags[1]) == owner and int(tb.tags[0]) == 0xFFFFFFFFFFFFFFFF
        n_owner = 5 if owner == 24 else 20
        assert st["conflicts"] == 25 - n_owner and st["tag_claims"] == 1
        want = [sq_leaf[1]] if owner == 24 else [sq_leaf[0], sq_leaf[2]]   # first reached first
        assert [x for x in tb.slots[1].tolist() if x != NONE32] == want


def test_first_epoch_length_hand_case():
    # 30 rays of one key (8) towards the three squares.  With epochs of 30 the
    # table is empty for all of them; with a first epoch of 3 rays (one per
    # square) the other 27 find all three leaves and are predicted, each by the
    # leaf of its own square (the other two boxes miss it).
    tris, b, sq_leaf = _three_squares()
    squares = np.array([2, 0, 1] * 10)
    rays = _rays_to_squares([-0.5, 1.0, 0.1], squares, 50)
    tb = oracle.Table(4, 4, 1, 1)
    _, st = oracle.trace(b, tris, rays, query="closest", mode="paper", table=tb, epoch=30)
    assert (st["positives"], st["pred_hits"], st["records"]) == (0, 0, 30)
    tb = oracle.Table(4, 4, 1, 1)
    hp, st = oracle.trace(b, tris, rays, query="closest", mode="paper", table=tb, epoch=30, first_epoch=3)
    assert (st["positives"], st["pred_hits"], st["records"], st["traversals"]) == (27, 27, 3, 3)
    e = int(np.nonzero(tb.tags != EMPTY_TAG)[0][0])
    assert sorted(x for x in tb.slots[e].tolist() if x != NONE32) == sorted(sq_leaf)
    exact, _ = oracle.trace(b, tris, rays, query="closest", mode="exact")
    assert np.array_equal(hp.view(np.uint32), exact.view(np.uint32))
    # a first epoch as long as the others is no first epoch at all
    t1, t2 = oracle.Table(4, 4, 1, 1), oracle.Table(4, 4, 1, 1)
    r1, s1 = oracle.trace(b, tris, rays, query="closest", mode="paper", table=t1, epoch=7, first_epoch=7)
    r2, s2 = oracle.trace(b, tris, rays, query="closest", mode="paper", table=t2, epoch=7)
    assert np.array_equal(r1.view(np.uint32), r2.view(np.uint32)) and s1 == s2
    assert np.array_equal(t1.tags, t2.tags) and np.array_equal(t1.slots, t2.slots)
    # longer than the other epochs: rejected
    with pytest.raises(ValueError):
        oracle.trace(b, tris, rays, query="closest", mode="paper", table=oracle.Table(4, 4, 1, 1), epoch=7,
                     first_epoch=8)


@pytest.mark.parametrize("first,epoch", [(1, 256), (100, 256), (256, 1000), (1000, 1000), (37, 4096)])
def test_first_epoch_equals_a_split_call(first, epoch):
    # epochs are boundaries in ray order, each seeing the table the earlier
    # ones left, with ray ids relative to the call: a call whose first epoch is
    # F rays long computes what a call of its first F rays (one epoch) followed
    # by a call of the rest (epochs of E) computes
    tris, rays = sg.tiny_workload()
    b = oracle.build_sah(tris)
    for query, mode in (("any", "paper"), ("closest", "paper"), ("closest", "exact")):
        r = rays.copy()
        if query == "closest":
            r[:, 7] = np.inf
        t1, t2 = oracle.Table(8, 4, 5, 6), oracle.Table(8, 4, 5, 6)
        a1, s1 = oracle.trace(b, tris, r, query=query, mode=mode, table=t1, epoch=epoch, first_epoch=first)
        a2, s2a = oracle.trace(b, tris, r[:first], query=query, mode=mode, table=t2, epoch=first)
        a3, s2b = oracle.trace(b, tris, r[first:], query=query, mode=mode, table=t2, epoch=epoch)
        both = np.concatenate([a2, a3])
        if query == "any":
            assert np.array_equal(a1, both)
        else:
            assert np.array_equal(a1.view(np.uint32), both.view(np.uint32))
        assert s1 == {k: s2a[k] + s2b[k] for k in s1}
        assert np.array_equal(t1.tags, t2.tags) and np.array_equal(t1.slots, t2.slots)


# ---------------------------------------------------------------------------
# The paper's IEEE-754 bit hash (hash_mode 1)
# ---------------------------------------------------------------------------

def test_paper_hash_hand_cases():
    rows = []
    with open(os.path.join(GOLDEN, "paper_hash_cases.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append(line.split())
    assert len(rows) == 2
    for row in rows:
        p = int(row[0])
        o = [float(x) for x in row[1:4]]
        d = [float(x) for x in row[4:7]]
        key = int(row[13])
        keys, idx = oracle.hash_rays(np.zeros(6, np.float32), p, p, 20, _ray(o, d), hash_mode=1)
        assert int(keys[0]) == key
        # the fold into the table is the same multiplicative hash as for the grid key
        k0, i0 = int(keys[0]), int(idx[0])
        assert i0 == ((k0 * 0x9E3779B97F4A7C15) % (1 << 64)) >> (64 - 20)


def test_paper_hash_bit_fields_and_width():
    g = np.random.default_rng(77)
    for p in range(1, 8):
        o = g.normal(size=(200, 3)).astype(np.float32) * 10
        d = g.normal(size=(200, 3)).astype(np.float32)
        rays = np.concatenate([o, np.zeros((200, 1)), d, np.ones((200, 1))], 1).astype(np.float32)
        keys, _ = oracle.hash_rays(np.zeros(6, np.float32), p, p, 16, rays, hash_mode=1)
        stride = 8 if p <= 3 else 16
        mask = (1 << (2 * p + 1)) - 1
        for k in keys[:50]:
            k = int(k)
            assert k < (1 << (3 * stride)) and k < (1 << 48)
            for f in range(3):
                assert (k >> (f * stride)) & ~mask & ((1 << stride) - 1) == 0   # 2p+1 bits per field
        # a sign flip of o.x flips exactly the top bit of field 0
        r2 = rays.copy()
        r2[:, 0] = -r2[:, 0]
        k2, _ = oracle.hash_rays(np.zeros(6, np.float32), p, p, 16, r2, hash_mode=1)
        assert all(int(a) ^ int(b) == (1 << (2 * p)) for a, b in zip(keys, k2))
        # similar rays (same exponent and leading mantissa bits) share a key
        r3 = rays.copy()
        r3[:, 0] = np.nextafter(r3[:, 0], np.float32(np.inf), dtype=np.float32)
        k3, _ = oracle.hash_rays(np.zeros(6, np.float32), p, p, 16, r3, hash_mode=1)
        same = np.count_nonzero(keys == k3)
        assert same >= 190


def test_paper_hash_trace_runs_and_keeps_invariants():
    tris = sg.triangle_soup(1, 256)
    rays = sg.tiny_shadow_rays(1, 4096)
    b = oracle.build_sah(tris)
    for p in (2, 4, 6):
        tb = oracle.Table(12, 4, p, p, hash_mode=1)
        out = np.zeros(4096, np.uint8)
        occ, st = oracle.trace(b, tris, rays, table=tb, epoch=256, outcome=out)
        _allowed_mismatch(tris, rays, occ != oracle.brute_force(tris, rays))
        _check_table_invariants(tb, set(int(x) for x in b.leaf_ids()))
        assert np.all(oracle.brute_force(tris, rays)[out == 2] == 1)
    with pytest.raises(ValueError):
        oracle.trace(b, tris, rays, table=oracle.Table(12, 4, 8, 8, hash_mode=1), epoch=256)


# ---------------------------------------------------------------------------
# Go Up Level (slots name the node g levels above the result leaf)
# ---------------------------------------------------------------------------

def _parents(b):
    par = np.full(b.num_nodes, NONE32, np.int64)
    for i in range(b.num_nodes):
        if b.right[i] != NONE32:
            par[i + 1] = i
            par[int(b.right[i])] = i
    return par


def _ancestor(par, node, g):
    for _ in range(g):
        if par[node] == NONE32:
            break
        node = int(par[node])
    return node


def test_go_up_hand_tree_slots_and_counters():
    # root(0) -> [inner(1) -> leaf A(2), leaf C(3)], leaf B(4); two identical
    # rays down onto A, one epoch per ray: ray 0 traverses and records, ray 1
    # is predicted
    tris = np.concatenate([_square(0, 0, 0), _square(0, 0, -1), _square(2, 0, 0)])
    b = _hand_bvh(tris, [(4, 0, 0, 0), (3, 0, 0, 1), (NONE32, 0, 2, 2), (NONE32, 2, 2, 2), (NONE32, 4, 2, 1)])
    down = _ray([0.75, 1, 0.25], [0, -1, 0])
    rays = np.stack([down, down])
    plain = dict(box_tests=5, nodes_visited=3, interior_visited=2, leaf_visited=1, tri_tests=1)
    for g, slot, pred in ((0, 0 << 3 | 1, dict(box_tests=1, nodes_visited=1, interior_visited=0, leaf_visited=1,
                                                 tri_tests=1, skipped=2)),
                          # parent of A: test node 1's box, then node 1 (A and C both hit, A nearer), A
                          (1, 1, dict(box_tests=3, nodes_visited=2, interior_visited=1, leaf_visited=1,
                                      tri_tests=1, skipped=1)),
                          # the root: the walk is the whole traversal, nothing skipped
                          (2, 0, dict(box_tests=5, nodes_visited=3, interior_visited=2, leaf_visited=1,
                                      tri_tests=1, skipped=0)),
                          (9, 0, dict(box_tests=5, nodes_visited=3, interior_visited=2, leaf_visited=1,
                                      tri_tests=1, skipped=0))):
        tb = oracle.Table(4, 2, 3, 3, go_up=g)
        out = np.zeros(2, np.uint8)
        occ, st = oracle.trace(b, tris, rays, table=tb, epoch=1, outcome=out)
        assert occ.tolist() == [1, 1] and out.tolist() == [1, 2]
        used = np.nonzero(tb.tags != EMPTY_TAG)[0]
        assert len(used) == 1 and tb.slots[used[0]].tolist() == [slot, NONE32]
        for k in ("box_tests", "nodes_visited", "interior_visited", "leaf_visited", "tri_tests"):
            assert st[k] == plain[k] + pred[k], (g, k)
        assert st["nodes_skipped"] == pred["skipped"] and st["traversals"] == 1 and st["pred_hits"] == 1
        assert st["pred_box_tests"] == pred["box_tests"] and st["pred_leaf_visited"] == 1
        assert st["pred_tri_tests"] == 1
    # a ray onto B (depth 1): at go-up 1 its parent is the root
    onto_b = _ray([2.75, 1, 0.25], [0, -1, 0])
    tb = oracle.Table(4, 2, 3, 3, go_up=1)
    oracle.trace(b, tris, onto_b[None], table=tb, epoch=1)
    assert tb.slots[tb.tags != EMPTY_TAG][0].tolist() == [0, NONE32]


def test_go_up_records_name_ancestors_of_exact_hits():
    # one epoch, EXACT closest: every hitting ray records the leaf of its exact
    # closest triangle (brute force), mapped g levels up; the table must be
    # what the update rule makes of those records, rebuilt here from scratch
    tris = sg.triangle_soup(5, 300, edge=0.12)
    g0 = np.random.default_rng(5)
    o = np.tile([[0.5, -0.5, 0.5]], (3000, 1)) + g0.uniform(-0.1, 0.1, (3000, 3))
    d = np.tile([[0.0, 1.0, 0.0]], (3000, 1)) + g0.uniform(-0.4, 0.4, (3000, 3))
    rays = sg.pack_rays(o.astype(np.float32), d.astype(np.float32), 0.0, np.inf)
    b = oracle.build_sah(tris)
    par = _parents(b)
    leaf_node_of_pos = {}
    for i in np.nonzero(b.right == NONE32)[0]:
        for k in range(int(b.first[i]), int(b.first[i] + b.count[i])):
            leaf_node_of_pos[k] = int(i)
    pos_of_prim = {int(p): k for k, p in enumerate(b.perm)}
    exact = oracle.brute_force(tris, rays, closest=True)
    T, W = 6, 3
    keys, idx = oracle.hash_rays(b.box[0], 3, 3, T, rays)
    for g in (1, 2, 3, 40):
        tb = oracle.Table(T, W, 3, 3, go_up=g)
        _, st = oracle.trace(b, tris, rays, query="closest", mode="exact", table=tb, epoch=rays.shape[0])
        want_tags = np.full(1 << T, EMPTY_TAG, np.uint64)
        want_slots = np.full((1 << T, W), NONE32, np.uint32)
        groups = {}
        for r in range(rays.shape[0]):
            prim = int(exact[r, 3].view(np.uint32))
            if prim != NONE32:
                node = _ancestor(par, leaf_node_of_pos[pos_of_prim[prim]], g)
                groups.setdefault(int(idx[r]), []).append((r, int(keys[r]), node))
        drops = conflicts = 0
        for i, recs in groups.items():
            kstar = recs[0][1]
            fresh = list(dict.fromkeys(n for _, k, n in recs if k == kstar))   # first record first
            want_tags[i] = kstar
            want_slots[i, :min(W, len(fresh))] = fresh[:W]
            drops += sum(1 for _, k, n in recs if k == kstar and n not in fresh[:W])
            conflicts += sum(1 for _, k, _n in recs if k != kstar)
        assert np.array_equal(tb.tags, want_tags), g
        assert np.array_equal(tb.slots, want_slots), g
        assert st["dropped"] == drops and st["conflicts"] == conflicts and st["tag_claims"] == len(groups)
        if g == 40:
            assert set(tb.slots[tb.tags != EMPTY_TAG][:, 0].tolist()) == {0}


def test_go_up_root_walk_equals_plain_traversal():
    # with every slot naming the root, a positive ray's walk is exactly the
    # plain traversal: its counts are the plain ones (without the traversal
    # count); a false positive then traverses again
    tris, rays, b, tb, _, _, _ = _config1(4096, table=oracle.Table(12, 4, 5, 6, go_up=64))
    assert set(tb.slots[tb.tags != EMPTY_TAG][:, 0].tolist()) == {0}
    out = np.zeros(rays.shape[0], np.uint8)
    occ, st = oracle.trace(b, tris, rays, table=tb, epoch=4096, outcome=out)
    assert np.array_equal(occ, oracle.brute_force(tris, rays))
    _, p_all = oracle.trace(b, tris, rays)
    _, p_fp = oracle.trace(b, tris, rays[out == 3])
    _, p_pos = oracle.trace(b, tris, rays[(out == 2) | (out == 3)])
    for k in ("box_tests", "nodes_visited", "interior_visited", "leaf_visited", "tri_tests"):
        assert st[k] == p_all[k] + p_fp[k], k
    assert st["pred_box_tests"] == p_pos["box_tests"]
    assert st["pred_leaf_visited"] == p_pos["leaf_visited"] and st["pred_tri_tests"] == p_pos["tri_tests"]
    assert st["pred_hits"] == np.count_nonzero(out == 2) > 100 and st["nodes_skipped"] == 0
    assert np.all(occ[out == 2] == 1) and np.all(occ[out == 3] == 0)
    assert st["traversals"] == np.count_nonzero((out == 1) | (out == 3))


@pytest.mark.parametrize("g", [1, 2, 3])
def test_go_up_results_and_invariants(g):
    tris = sg.triangle_soup(1, 256)
    rays = sg.tiny_shadow_rays(1, 4096)
    b = oracle.build_sah(tris)
    par = _parents(b)
    valid = {_ancestor(par, int(i), g) for i in np.nonzero(b.right == NONE32)[0]}
    tb = oracle.Table(12, 4, 5, 6, go_up=g)
    occ, st = oracle.trace(b, tris, rays, table=tb, epoch=256)
    _allowed_mismatch(tris, rays, occ != oracle.brute_force(tris, rays))
    _check_table_invariants(tb, valid)
    assert st["pred_hits"] > 0
    # closest: EXACT equals brute force; PAPER accepts only real hits
    rc = rays.copy()
    rc[:, 7] = np.inf
    he = oracle.brute_force(tris, rc, closest=True)
    hx, _ = oracle.trace(b, tris, rc, query="closest", mode="exact", table=oracle.Table(12, 4, 5, 6, go_up=g),
                         epoch=256)
    assert np.array_equal(hx[:, 3].view(np.uint32), he[:, 3].view(np.uint32))
    hp, sp = oracle.trace(b, tris, rc, query="closest", mode="paper", table=oracle.Table(12, 4, 5, 6, go_up=g),
                          epoch=256)
    hit = hp[:, 3].view(np.uint32) != NONE32
    assert np.array_equal(hit, he[:, 3].view(np.uint32) != NONE32)
    for r in np.nonzero(hit)[0][:300]:
        h, t, _, _ = oracle.mt(tris[hp[r, 3].view(np.uint32)], rc[r])
        assert h and t == hp[r, 0]
    with pytest.raises(ValueError):
        oracle.trace(b, tris, rays, table=oracle.Table(12, 4, 5, 6, go_up=65), epoch=256)


def _subtree_ranges(b):
    lo = np.zeros(b.num_nodes, np.int64)
    hi = np.zeros(b.num_nodes, np.int64)

    def rec(i):
        if b.right[i] == NONE32:
            lo[i], hi[i] = int(b.first[i]), int(b.first[i] + b.count[i])
        else:
            rec(i + 1)
            rec(int(b.right[i]))
            lo[i] = min(lo[i + 1], lo[int(b.right[i])])
            hi[i] = max(hi[i + 1], hi[int(b.right[i])])
    rec(0)
    return lo, hi


@pytest.mark.parametrize("g", [1, 3])
def test_go_up_exact_prediction_hits_by_subtree_membership(g):
    # EXACT closest: a positive ray counts a prediction hit iff its exact
    # closest triangle lies in the subtree of one of the entry's nodes; the
    # table is frozen for the second call (one epoch), so every decision can
    # be recomputed here from the snapshot
    tris = sg.triangle_soup(7, 300, edge=0.12)
    g0 = np.random.default_rng(7)
    o = np.tile([[0.5, -0.5, 0.5]], (3000, 1)) + g0.uniform(-0.1, 0.1, (3000, 3))
    d = np.tile([[0.0, 1.0, 0.0]], (3000, 1)) + g0.uniform(-0.4, 0.4, (3000, 3))
    rays = sg.pack_rays(o.astype(np.float32), d.astype(np.float32), 0.0, np.inf)
    b = oracle.build_sah(tris)
    lo, hi = _subtree_ranges(b)
    pos_of_prim = {int(p): k for k, p in enumerate(b.perm)}
    T = 8
    tb = oracle.Table(T, 4, 4, 4, go_up=g)
    oracle.trace(b, tris, rays, query="closest", mode="exact", table=tb, epoch=rays.shape[0])
    snap = tb.copy()
    out = np.zeros(rays.shape[0], np.uint8)
    _, st = oracle.trace(b, tris, rays, query="closest", mode="exact", table=tb, epoch=rays.shape[0], outcome=out)
    exact = oracle.brute_force(tris, rays, closest=True)
    keys, idx = oracle.hash_rays(b.box[0], 4, 4, T, rays)
    want_hits = want_fp = 0
    for r in range(rays.shape[0]):
        i = int(idx[r])
        slots = [int(x) for x in snap.slots[i] if x != NONE32]
        if not (snap.tags[i] == keys[r] and slots):
            assert out[r] == 1
            continue
        prim = int(exact[r, 3].view(np.uint32))
        inside = prim != NONE32 and any(lo[n] <= pos_of_prim[prim] < hi[n] for n in slots)
        want_hits += inside
        want_fp += not inside
        assert out[r] == (2 if inside else 3)
    assert st["pred_hits"] == want_hits > 50 and st["false_pos"] == want_fp > 0


# ---------------------------------------------------------------------------
# Replacement policies (bit 0: FIFO eviction within an entry; bit 1: the
# resident tag keeps its entry)
# ---------------------------------------------------------------------------

def test_fifo_eviction_hand_case():
    # one key (8), W = 2; epoch 1 reaches square 0, epoch 2 squares 1 and 2,
    # epoch 3 square 0 again (each call is one epoch)
    tris, b, sq_leaf = _three_squares()
    r0 = _rays_to_squares([-0.5, 1.0, 0.1], np.array([0] * 6), 60)
    # square 2 is reached first: its leaf (the larger id) goes first
    r12 = _rays_to_squares([-0.5, 1.0, 0.1], np.array([2, 1] * 5), 61)
    first, second = sq_leaf[2], sq_leaf[1]
    for policy in (0, 1):
        tb = oracle.Table(4, 2, 1, 1, policy=policy)
        oracle.trace(b, tris, r0, query="closest", mode="exact", table=tb, epoch=1000)
        e = int(np.nonzero(tb.tags != EMPTY_TAG)[0][0])
        assert tb.slots[e].tolist() == [sq_leaf[0], NONE32]
        _, st = oracle.trace(b, tris, r12, query="closest", mode="exact", table=tb, epoch=1000)
        if policy == 0:
            # no eviction: one free slot takes the first reached new leaf, the other is dropped
            assert tb.slots[e].tolist() == [sq_leaf[0], first]
            assert (st["leaf_inserts"], st["evictions"], st["dropped"]) == (1, 0, 5)
        else:
            # FIFO: the oldest leaf (square 0) leaves, both new leaves enter in ray order
            assert tb.slots[e].tolist() == [first, second]
            assert (st["leaf_inserts"], st["evictions"], st["dropped"]) == (2, 1, 0)
        _, st = oracle.trace(b, tris, r0, query="closest", mode="exact", table=tb, epoch=1000)
        if policy == 1:
            assert tb.slots[e].tolist() == [second, sq_leaf[0]]
            assert (st["leaf_inserts"], st["evictions"]) == (1, 1)
        else:
            assert tb.slots[e].tolist() == [sq_leaf[0], first] and st["leaf_inserts"] == 0


def test_resident_tag_keeps_its_entry_hand_case():
    # keys 8 (rays from above) and 24 (from below) share index 1 of a 2-entry table
    tris, b, sq_leaf = _three_squares()
    below = _rays_to_squares([-0.5, -1.0, 0.1], np.array([1] * 5), 53)
    above = _rays_to_squares([-0.5, 1.0, 0.1], np.array([0, 2] * 10), 54)
    for policy in (0, 2):
        tb = oracle.Table(1, 4, 1, 1, policy=policy)
        oracle.trace(b, tris, above, query="closest", mode="exact", table=tb, epoch=100)
        assert int(tb.tags[1]) == 8
        resident = tb.slots[1].copy()
        _, st = oracle.trace(b, tris, below, query="closest", mode="exact", table=tb, epoch=100)
        if policy == 0:
            # the smallest ray id's key (24) takes the entry over
            assert int(tb.tags[1]) == 24 and tb.slots[1].tolist() == [sq_leaf[1], NONE32, NONE32, NONE32]
            assert (st["tag_claims"], st["conflicts"]) == (1, 0)
        else:
            # the resident key 8 keeps it; key 24's records are conflicts
            assert int(tb.tags[1]) == 8 and np.array_equal(tb.slots[1], resident)
            assert (st["tag_claims"], st["conflicts"], st["leaf_inserts"]) == (0, 5, 0)
    # an empty entry is still claimed by the smallest ray id's key
    tb = oracle.Table(1, 4, 1, 1, policy=2)
    oracle.trace(b, tris, np.concatenate([below, above]), query="closest", mode="exact", table=tb, epoch=100)
    assert int(tb.tags[1]) == 24


@pytest.mark.parametrize("policy", [1, 2, 3])
def test_policies_results_invariants_and_special_cases(policy):
    tris = sg.triangle_soup(1, 256)
    rays = sg.tiny_shadow_rays(1, 4096)
    b = oracle.build_sah(tris)
    valid = set(int(x) for x in b.leaf_ids())
    for T, W in ((4, 2), (8, 1), (12, 4)):
        tb = oracle.Table(T, W, 5, 6, policy=policy)
        out = np.zeros(4096, np.uint8)
        occ, st = oracle.trace(b, tris, rays, table=tb, epoch=256, outcome=out)
        _allowed_mismatch(tris, rays, occ != oracle.brute_force(tris, rays))
        _check_table_invariants(tb, valid)
        assert np.all(oracle.brute_force(tris, rays)[out == 2] == 1)
        if policy & 1:
            assert st["evictions"] <= st["leaf_inserts"]
        else:
            assert st["evictions"] == 0
        if policy == 3:
            # no tag is ever replaced, so every slot in use is an insert not yet evicted
            assert np.count_nonzero(tb.slots != NONE32) == st["leaf_inserts"] - st["evictions"]
    # special cases that reduce to the rule without eviction: FIFO never evicts
    # when entries are wide enough, and the resident rule never differs when no
    # two keys share an index
    base = oracle.Table(20, 8, 5, 6)
    _, s0 = oracle.trace(b, tris, rays, table=base, epoch=256)
    assert s0["dropped"] == 0 and s0["conflicts"] == 0
    tb = oracle.Table(20, 8, 5, 6, policy=policy)
    _, s1 = oracle.trace(b, tris, rays, table=tb, epoch=256)
    assert s1 == s0 and np.array_equal(tb.slots, base.slots) and np.array_equal(tb.tags, base.tags)
    with pytest.raises(ValueError):
        oracle.trace(b, tris, rays, table=oracle.Table(12, 4, 5, 6, policy=4), epoch=256)
