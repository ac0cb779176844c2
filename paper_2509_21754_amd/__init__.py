"""MI355X (gfx950) FITrig trigger: HIP kernels behind a C ABI (include/fitrig.h).

The Python side only marshals arguments; see ``fitrig.py``.
"""
from .fitrig import (  # noqa: F401
    Context, FitrigError, Server, fitrig_abi_version, fitrig_config_default, fitrig_create, fitrig_destroy,
    fitrig_detect, fitrig_interp_peaks, fitrig_last_hip_error, fitrig_phase_times, fitrig_status_string,
    interp_peaks, load, accumulate, accum_factor, fitrig_accumulate, fitrig_accum_factor, fitrig_index_prefix, index_prefix, INTERP_BILINEAR, INTERP_BICUBIC, INTERP_SPLINE, INTERP_MAKIMA,
)
