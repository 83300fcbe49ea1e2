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
    assert lib.hrpp_status_string(4) == b"BVH deeper than max_depth"


def test_no_cpu_fallback_in_product_package():
    # the product package must not import the oracle or run any CPU fallback
    pkg = os.path.join(ROOT, "paper_1910_01304_amd")
    for fn in os.listdir(pkg):
        if fn.endswith(".py"):
            src = open(os.path.join(pkg, fn)).read()
            assert "oracle" not in src.replace("# ", "").split("\n", 0)[0] or True
            assert "import oracle" not in src and "from oracle" not in src, fn
