"""MI355X-native recursive multiscale Robin coupled method (MRCM).

The product is the C-ABI shared library ``librmrcm.so`` built from
``csrc/`` (HIP kernels for gfx950 plus the host runtime); ``rmrcm`` is its
Python binding.  There is no CPU fallback: without the built library the
binding raises on first use.
"""

from .rmrcm import (  # noqa: F401
    Solver,
    Batch,
    Net,
    rmrcm_export_local,
    rmrcm_get_gate,
    rmrcm_plan_bytes,
    rmrcm_set_refinement,
    rmrcm_downscale,
    rmrcm_autotune,
    RMRCMError,
    load_library,
    rmrcm_default_params,
    rmrcm_setup,
    rmrcm_refactor,
    rmrcm_sync,
    rmrcm_solve,
    rmrcm_step_noalloc,
    rmrcm_get_interface,
    rmrcm_counts,
    rmrcm_set_stream,
    rmrcm_get_stats,
    rmrcm_destroy,
    rmrcm_strerror,
    RMRCM_FP64,
    RMRCM_MIXED,
    RMRCM_MIXED_LEARNED,
    EXPORTS,
)
