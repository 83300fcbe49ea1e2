"""MI355X-native Hash-Based Ray Path Prediction (HRPP).

The compute path is the HIP library ``libhrpp.so`` (include/hrpp.h); this
package is its Python binding.
"""
from .hrpp import (  # noqa: F401
    BVH, Predictor, HrppError, STAT_NAMES, SCHEDULE_STATS, EXPORTED, load_library, new_stats, stats_dict, trace_anyhit,
    trace_closest, trace_wide_anyhit, trace_wide_closest, get_error, LIB_PATH, profile_start, profile_stop, Batch,
    profile_touch, TOUCH_KINDS, TOUCH_REGIONS,
    Server,
)
