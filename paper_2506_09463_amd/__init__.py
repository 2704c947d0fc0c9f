"""MI355X-native in-place Householder QR least squares (libhqr, gfx950).

The compute path is the HIP library ``libhqr.so`` (C ABI in include/hqr.h);
``hqr`` is its thin ctypes binding.  Nothing in this package falls back to a
CPU implementation.
"""
from .hqr import (  # noqa: F401
    EXPORTS, HQR_EDEVICE, HQR_ENOMEM, HQR_ENOTSUP, HQR_INFO_NOCONV, HQR_INFO_TIMEOUT,
    HQR_OPT_NO_FALLBACK, HQR_OPT_TSQR_PANEL, HQR_PREC_FP64, HQR_PREC_MIXED, HQR_TUNE_BATCHED, HQR_TUNE_OCCUPANCY, HQR_TUNE_SINGLE, HQRError, colmajor, empty_colmajor, load,
    load_tune_db, tune_clear, tune_set, tune_variants, variant_shape,
    BatchPlan, batched_workspace_size, chol_update, cholesky, profile_begin, profile_end, qr_apply_q, qr_apply_qt, qr_backsolve, qr_factor, qr_form_q,
    qr_lse_solve, qr_lsq_refine, qr_lsq_solve, qr_lsq_solve_batched,
    status_string, version,
    workspace_size, workspace_size_opts,
)
