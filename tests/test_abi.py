"""CPU-side checks of the C-ABI library: it loads, exports every declared
entry point, validates arguments on the host, and its host BVH builder
reproduces the oracle's tree bit for bit."""
from __future__ import annotations

import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
import scenegen as sg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hrpp.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(hrpp_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    hrpp = pytest.importorskip("paper_1910_01304_amd")
    lib_path = hrpp.LIB_PATH
    assert os.path.exists(lib_path), "libhrpp.so not built"
    out = subprocess.check_output(["nm", "-D", "--defined-only", lib_path], text=True)
    exported = set(re.findall(r" T (hrpp_[a-z_0-9]+)$", out, re.M))
    declared = _declared()
    assert len(declared) >= 19
    missing = [s for s in declared if s not in exported]
    assert not missing, missing
    assert set(hrpp.EXPORTED) <= exported
    lib = hrpp.load_library()
    for s in declared:
        assert hasattr(lib, s)


def test_host_builder_matches_oracle_bit_for_bit():
    hrpp = pytest.importorskip("paper_1910_01304_amd")
    cases = [sg.triangle_soup(1, 256), sg.triangle_soup(2, 5), sg.triangle_soup(3, 1),
             np.repeat(sg.triangle_soup(4, 1), 40, axis=0), sg.scaled_terrain_scene(5, 20000)[0]]
    for tris in cases:
        for leaf_max, bins in ((4, 32), (2, 8), (8, 16)):
            b = hrpp.BVH(tris, leaf_max=leaf_max, sah_bins=bins, device=None)
            e = b.export()
            o = oracle.build_sah(tris, leaf_max=leaf_max, bins=bins)
            for k in ("box", "right", "first", "count", "depth", "perm"):
                assert np.array_equal(e[k].view(np.uint32), getattr(o, k).view(np.uint32)), k
            assert b.max_depth == o.max_depth()
            oracle.validate_bvh(o, tris, leaf_max, 64)


def test_host_treelet_passes_match_oracle_bit_for_bit():
    # the SAH tree after treelet restructuring (host C++) against the oracle's
    hrpp = pytest.importorskip("paper_1910_01304_amd")
    cases = [sg.triangle_soup(11, 7), sg.triangle_soup(12, 300), np.repeat(sg.triangle_soup(4, 1), 40, axis=0),
             sg.scaled_terrain_scene(5, 20000)[0]]
    for tris in cases:
        for leaf_max, passes in ((1, 1), (2, 2), (4, 3)):
            b = hrpp.BVH(tris, leaf_max=leaf_max, device=None, treelet_passes=passes)
            e = b.export()
            o = oracle.build_sah(tris, leaf_max=leaf_max, treelet_passes=passes)
            for k in ("box", "right", "first", "count", "depth", "perm"):
                assert np.array_equal(e[k].view(np.uint32), getattr(o, k).view(np.uint32)), (k, passes)
            assert b.max_depth == o.max_depth()
            oracle.validate_bvh(o, tris, leaf_max, 64)


def test_host_argument_validation():
    hrpp = pytest.importorskip("paper_1910_01304_amd")
    lib = hrpp.load_library()
    tris = sg.triangle_soup(1, 16)
    v = np.ascontiguousarray(tris.reshape(-1, 9))
    desc = hrpp.hrpp._BvhDesc(4, 32, 64)
    h = C.c_void_p()
    assert lib.hrpp_bvh_build_host(None, 16, C.byref(desc), C.byref(h)) == 1
    assert lib.hrpp_bvh_build_host(v.ctypes.data, 0, C.byref(desc), C.byref(h)) == 1
    bad = hrpp.hrpp._BvhDesc(9, 32, 64)
    assert lib.hrpp_bvh_build_host(v.ctypes.data, 16, C.byref(bad), C.byref(h)) == 1
    vnan = v.copy()
    vnan[3, 4] = np.nan
    assert lib.hrpp_bvh_build_host(vnan.ctypes.data, 16, C.byref(desc), C.byref(h)) == 1
    # a chain too deep for max_depth reports EDEPTH
    same = np.ascontiguousarray(np.repeat(tris[:1], 64, axis=0).reshape(-1, 9))
    shallow = hrpp.hrpp._BvhDesc(1, 32, 3)
    assert lib.hrpp_bvh_build_host(same.ctypes.data, 64, C.byref(shallow), C.byref(h)) == 4
    # a host-only BVH cannot be traced: EINVAL before any device call
    assert lib.hrpp_bvh_build_host(v.ctypes.data, 16, C.byref(desc), C.byref(h)) == 0
    assert lib.hrpp_trace_anyhit(h, None, C.c_void_p(16), 4, C.c_void_p(16), None, None) == 1
    lib.hrpp_bvh_destroy(h)
    # the device build rejects null pointers, empty input, a bad descriptor and
    # misaligned buffers before any device call
    p16 = C.c_void_p(256)
    assert lib.hrpp_bvh_device_build_scratch_bytes(0) == 0
    assert lib.hrpp_bvh_device_build_scratch_bytes(1 << 28) == 0
    assert lib.hrpp_build_bvh_device(None, 16, C.byref(desc), p16, 1 << 20, p16, 1 << 20, None, C.byref(h)) == 1
    assert lib.hrpp_build_bvh_device(p16, 0, C.byref(desc), p16, 1 << 20, p16, 1 << 20, None, C.byref(h)) == 1
    assert lib.hrpp_build_bvh_device(p16, 16, C.byref(bad), p16, 1 << 20, p16, 1 << 20, None, C.byref(h)) == 1
    assert lib.hrpp_build_bvh_device(p16, 16, C.byref(shallow), None, 1 << 20, p16, 1 << 20, None, C.byref(h)) == 1
    assert lib.hrpp_build_bvh_device(p16, 16, C.byref(desc), C.c_void_p(260), 1 << 20, p16, 1 << 20, None,
                                     C.byref(h)) == 1
    assert lib.hrpp_build_bvh_device(p16, 16, C.byref(hrpp.hrpp._BvhDesc(4, 32, 65)), p16, 1 << 20, p16, 1 << 20,
                                     None, C.byref(h)) == 1
    assert lib.hrpp_build_bvh_device(p16, 16, C.byref(desc), p16, 1 << 20, p16, 1 << 20, None, None) == 1
    # treelet passes: at most 8
    assert lib.hrpp_build_bvh_device(p16, 16, C.byref(hrpp.hrpp._BvhDesc(4, 32, 64, 9)), p16, 1 << 20, p16, 1 << 20,
                                     None, C.byref(h)) == 1
    assert lib.hrpp_bvh_build_host(v.ctypes.data, 16, C.byref(hrpp.hrpp._BvhDesc(4, 32, 64, 9)), C.byref(h)) == 1
    idx = C.c_uint32()
    assert lib.hrpp_serve_add_scene(None, None, C.byref(idx)) == 1
    assert lib.hrpp_serve_remove_scene(None, 0) == 1
    # predictor descriptor limits
    pd = hrpp.hrpp._PredDesc(12, 4, 5, 6, 256, 0, 0)
    assert lib.hrpp_predictor_required_bytes(C.byref(pd)) > (1 << 12) * 32
    assert lib.hrpp_predictor_table_bytes(C.byref(pd)) == (1 << 12) * 32
    for badp in (hrpp.hrpp._PredDesc(0, 4, 5, 6, 256, 0, 0), hrpp.hrpp._PredDesc(12, 9, 5, 6, 256, 0, 0),
                 hrpp.hrpp._PredDesc(12, 4, 5, 6, 0, 0, 0), hrpp.hrpp._PredDesc(12, 4, 5, 6, 256, 2, 0),
                 # the bit-field hash: precision 1..7 and dir_bits equal to origin_bits
                 hrpp.hrpp._PredDesc(12, 4, 5, 6, 256, 1, 0), hrpp.hrpp._PredDesc(12, 4, 8, 8, 256, 1, 0),
                 hrpp.hrpp._PredDesc(12, 4, 0, 0, 256, 1, 0)):
        assert lib.hrpp_predictor_required_bytes(C.byref(badp)) == 0
    for p in range(1, 8):
        assert lib.hrpp_predictor_required_bytes(C.byref(hrpp.hrpp._PredDesc(12, 4, p, p, 256, 1, 0))) > 0
    # go-up levels 0..64
    assert lib.hrpp_predictor_required_bytes(C.byref(hrpp.hrpp._PredDesc(12, 4, 5, 6, 256, 0, 64))) > 0
    assert lib.hrpp_predictor_required_bytes(C.byref(hrpp.hrpp._PredDesc(12, 4, 5, 6, 256, 0, 65))) == 0
    # inline_lanes: 0 (default) .. 65 (always queue)
    assert lib.hrpp_predictor_required_bytes(C.byref(hrpp.hrpp._PredDesc(12, 4, 5, 6, 256, 0, 0, 65))) > 0
    assert lib.hrpp_predictor_required_bytes(C.byref(hrpp.hrpp._PredDesc(12, 4, 5, 6, 256, 0, 0, 66))) == 0
    # replacement policies 0..3
    assert lib.hrpp_predictor_required_bytes(C.byref(hrpp.hrpp._PredDesc(12, 4, 5, 6, 256, 0, 0, 0, 3))) > 0
    assert lib.hrpp_predictor_required_bytes(C.byref(hrpp.hrpp._PredDesc(12, 4, 5, 6, 256, 0, 0, 0, 4))) == 0
    # first epoch: 0 (= epoch_rays) .. epoch_rays
    for first, ok in ((0, True), (1, True), (256, True), (257, False)):
        need = lib.hrpp_predictor_required_bytes(C.byref(hrpp.hrpp._PredDesc(12, 4, 5, 6, 256, 0, 0, 0, 0, first)))
        assert (need > 0) == ok, first
    assert lib.hrpp_status_string(4) == b"BVH deeper than max_depth"


def test_no_cpu_fallback_in_product_package():
    # the product package must not import the oracle or run any CPU fallback
    pkg = os.path.join(ROOT, "paper_1910_01304_amd")
    for fn in os.listdir(pkg):
        if fn.endswith(".py"):
            src = open(os.path.join(pkg, fn)).read()
            assert "oracle" not in src.replace("# ", "").split("\n", 0)[0] or True
            assert "import oracle" not in src and "from oracle" not in src, fn


def _python_wide(e):
    """The 4-wide collapse written out from its definition (include/hrpp.h):
    start from a binary node's two children; while fewer than four, replace the
    interior child of largest half area (double; ties to the earlier child) by
    its two children, in place; number wide nodes in depth-first pre-order."""
    NONE = 0xFFFFFFFF
    box, right, first, count = e["box"], e["right"], e["first"], e["count"]
    words = []

    def area(i):
        b = box[i].astype(np.float64)
        dx, dy, dz = b[3] - b[0], b[4] - b[1], b[5] - b[2]
        return dx * dy + dy * dz + dz * dx

    def leaf_ref(i):
        return 0x80000000 | (int(first[i]) << 3) | (int(count[i]) - 1)

    def emit(i):
        ch = [i + 1, int(right[i])]
        while len(ch) < 4:
            inner = [k for k, c in enumerate(ch) if right[c] != NONE]
            if not inner:
                break
            k = max(inner, key=lambda k: (area(ch[k]), -k))
            c = ch[k]
            ch[k:k + 1] = [c + 1, int(right[c])]
        wid = len(words)
        words.append(np.zeros(32, np.uint32))
        for k in range(4):
            if k < len(ch):
                b = box[ch[k]].view(np.uint32)
                for a, comp in enumerate((0, 3, 1, 4, 2, 5)):
                    words[wid][4 * a + k] = b[comp]
                words[wid][24 + k] = leaf_ref(ch[k]) if right[ch[k]] == NONE else emit(ch[k])
            else:
                words[wid][24 + k] = NONE
        return wid

    if right[0] == NONE:
        return np.zeros((0, 32), np.uint32), leaf_ref(0)
    emit(0)
    return np.stack(words), 0


def test_wide_tree_matches_its_definition_and_is_valid():
    hrpp = pytest.importorskip("paper_1910_01304_amd")
    for tris in (sg.triangle_soup(1, 256), sg.triangle_soup(3, 1), sg.triangle_soup(2, 7),
                 sg.scaled_terrain_scene(5, 20000)[0]):
        for leaf_max in (1, 4):
            b = hrpp.BVH(tris, leaf_max=leaf_max, device=None)
            e = b.export()
            info = b.wide_info()
            words = b.wide_export()
            want, root = _python_wide(e)
            assert info["root_ref"] == root and np.array_equal(words, want)
            if root & 0x80000000:
                continue
            # every binary leaf exactly once; each node's box is the exact union of
            # its children's boxes; stack need and depth bound every traversal
            leaves = {(int(e["first"][i]) << 3) | (int(e["count"][i]) - 1)
                      for i in np.nonzero(e["right"] == 0xFFFFFFFF)[0]}
            seen = []

            def walk(n):
                refs = words[n, 24:28]
                nch = int(np.count_nonzero(refs != 0xFFFFFFFF))
                assert 2 <= nch <= 4 and np.all(refs[nch:] == 0xFFFFFFFF)
                need, depth = 0, 0
                for k in range(nch):
                    ref = int(refs[k])
                    if ref & 0x80000000:
                        seen.append(ref & 0x7FFFFFFF)
                    else:
                        cb = words[ref, 24:28]
                        m = cb != 0xFFFFFFFF
                        lo = [words[ref, 4 * a:4 * a + 4].view(np.float32)[m].min() for a in (0, 2, 4)]
                        hi = [words[ref, 4 * a:4 * a + 4].view(np.float32)[m].max() for a in (1, 3, 5)]
                        assert np.array_equal(np.array(lo + hi, np.float32),
                                              np.array([words[n, 4 * a + k].view(np.float32)
                                                        for a in (0, 2, 4, 1, 3, 5)], np.float32))
                        cn, cd = walk(ref)
                        need, depth = max(need, cn), max(depth, cd)
                return nch - 1 + need, depth + 1

            need, depth = walk(0)
            assert sorted(seen) == sorted(leaves)
            assert info["stack_need"] == need and info["depth"] == depth
