"""MI355X (gfx950) pseudo-spectral phase-field-crystal (PFC) hot path.

Python binding of ``libpfc.so`` (C ABI in ``include/pfc.h``).  This module only marshals
arguments: every transform, update and reduction runs in the library's HIP kernels.  PyTorch
provides device memory and streams.  There is no fallback: if the library is not built, importing
the binding raises.
"""
from __future__ import annotations

from ._binding import (  # noqa: F401
    PFC_F32,
    PFC_F64,
    PFC_FLAG_LINEAR_ONLY,
    PFC_ONE_MODE,
    PFC_TWO_MODE,
    Apfc,
    Batch,
    HydroParams,
    PfcError,
    Plan,
    library_path,
    load_library,
    pfc_apfc_create,
    pfc_apfc_fft,
    pfc_apfc_nonlinear,
    pfc_apfc_state_init,
    pfc_apfc_step,
    pfc_energy,
    pfc_fft_c2r,
    pfc_fft_r2c,
    pfc_hydro_state_init,
    pfc_hydro_step,
    pfc_plan_create,
    pfc_plan_destroy,
    pfc_plan_set_params,
    pfc_state_export,
    pfc_state_init,
    pfc_step,
    pfc_step_backward,
    pfc_step_timed,
)
from .rollout import PFCRollout, loss_and_grad  # noqa: F401,E402
