"""MI355X (gfx950) ultrafast power-Doppler reconstruction path.

RF synthesis -> RF-to-IQ + 3-D delay-and-sum with coherent compounding -> Casorati
Gram -> FP64 eigendecomposition and rank selection -> SVD clutter filter -> power
Doppler, plus a learned slow-time convolutional clutter filter with SVD fallback.
All stages are hand-written HIP kernels in libfqpd.so (C ABI: include/fqpd.h);
this package is the thin Python binding over it.
"""
from ._lib import (  # noqa: F401
    FQ_MAX_ANGLES, FQ_MAX_NT, FQ_SSM_MAX_MODES, LCF_N_PARAM, FqError, CUTOFF_KNEE, CUTOFF_SSM, DISP_POWER, DISP_IQ, MIP_XY, MIP_XZ, MIP_YZ,
    GRAM_FP32, GRAM_SPLIT_BF16, GRAM_BF16, GRAM_SPLIT4_BF16, INTERP_LINEAR, INTERP_HERMITE,
    Probe, Tx, Grid, Pulse, FdParams, make_probe, make_tx, make_grid, make_pulse, make_fd_params, lib,
    fd_workspace_size, fd_synth,
    rf_synth, das_workspace_size, das_window_rows, das_beamform, das_demodulate, das_delay_sum, gram_workspace_size, casorati_gram, casorati_gram_noalloc,
    svd_workspace_size, svd_clutter_filter, svd_filter_apply, hermitian_eig, power_doppler, ssm_workspace_size, spatial_similarity,
    display_workspace_size, display_db, mip, image_quality,
    lcf_act_size, lcf_forward, lcf_backward, lcf_adam_step, lcf_gather,
    fallback_workspace_size, lcf_fallback,
    roof_probe, PROBE_LDS_READ, PROBE_FP32_FMA,
    fq_workspace_size, WS_DAS, WS_DAS_MIN, WS_GRAM, WS_SVD, WS_SSM, WS_FD, WS_DISPLAY, WS_FALLBACK, WS_LCF_ACT,
)
