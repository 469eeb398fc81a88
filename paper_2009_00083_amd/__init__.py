"""MI355X-native critical-point classification of PL scalar fields on grids.

The classification (Section 3.1 of Lukasczyk et al., "Localized Topological
Simplification of Scalar Data", with the index tie-break of Section 4.1) runs
in the HIP kernels of ``libpcrit.so``; this package only marshals arguments
to its C ABI (``include/pcrit.h``).  PyTorch supplies device memory and
streams.  There is no CPU fallback: if the library is missing, every call
raises.
"""
from .binding import (  # noqa: F401
    PcritError, Context, classify, classify_noalloc, classify_batch, BatchResult, order_field, extrema, lts_propagate, lts_merged, batch_autotune, progressive, progressive_async, max_level, level_dims,
    link_table, preview_f1, preview_f1_levels, library_path, decode, is_critical, point_type,
    region_count, mlp_feature_level, mlp_features, mlp_labels, mlp_forward, mlp_backward,
    mlp_adam, progressive_timeline, MLP_PARAMS, MLP_INPUTS,
    E_ARG, E_DIMS, E_LEVEL, E_CAPACITY, E_NAN, E_HIP, E_OOM, E_SCRATCH,
    NOALLOC_SCRATCH_BYTES, LTS_SADDLE, LTS_PERSISTENT, LTS_BUDGET, LTS_INVALID,
    LTS_MAX_VISITED, LTS_MAX_FRONTIER,
)
from . import learned_order  # noqa: F401,E402
