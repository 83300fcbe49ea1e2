"""CPU oracle for Hash-Based Ray Path Prediction -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps ``hrpp_oracle.c`` (plain C, binary32 ops in a
fixed order, OpenMP across the rays of one epoch) and adds the fp64 and
validation helpers the pins use.  It shares no code with the GPU library.
"""
from .core import (  # noqa: F401
    STAT_NAMES, CanonBVH, Table, build_sah, build_median, build_lbvh, lbvh_codes, bvh_vertices, trace, brute_force,
    hash_rays, mt, slab, lib_path, build_library,
)
from .validate import validate_bvh  # noqa: F401
