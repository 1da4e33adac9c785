"""MI355X nested-mesh dynamical-friction solver (Velasco Romero & Masset 2018).

Thin Python binding of the C ABI in ``include/df.h`` (``libdfmesh.so``, HIP
kernels for gfx950).  PyTorch supplies only the device arena and the stream;
every step of the update runs in the library's kernels.  There is no CPU
fallback: importing this package without the built library raises.
"""
from ._lib import (  # noqa: F401
    DF_FP32, DF_FP64, FIELDS, KERNEL_KINDS, DFError, Engine, Run, bind, debug_stage, destroy,
    engine_job_bytes, force, force_density,
    force_log, get_dt, get_field, init_mesh, lib_path, required_bytes, set_field, set_perturber,
    step, stream_copy, sync_levels, timing_enable, timing_read, totals,
)
