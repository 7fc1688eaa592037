"""MI355X-native Smith-Waterman-Gotoh alignment (the SSW method's hot path).

Thin ctypes binding over the C-ABI library ``libswx.so`` (see
``include/swx.h``).  Every step of the alignment runs in the library's HIP
kernels; this module only marshals arguments.  Importing it does not load the
library; the first call does, and fails loudly when the library is missing.
"""
from ._binding import (  # noqa: F401
    SWX_ALL, SWX_BEGIN, SWX_CIGAR, SWX_SCORE2, SWX_SUBOPT, SWX_MEM_DEVICE, SWX_MEM_HOST, SWX_REF_DEVICE,
    Context, SwxError, decode_cigar, lib, lib_path, swx_align, swx_align_batch,
    swx_align_batch_noalloc, swx_cigar_bound,
    swx_ctx_create, swx_ctx_destroy, swx_last_error, swx_last_stage_ms, swx_profile_create,
    swx_profile_destroy, swx_result_free, swx_strerror, swx_get_tuning, swx_set_tuning, REC_DTYPE,
    Server, make_requests, REQ_DTYPE, COMPLETION_DTYPE, SWX_EBUSY, Graph,
    simulate_serving, SIM_REQ_DTYPE, SIM_RESULT_DTYPE,
)
