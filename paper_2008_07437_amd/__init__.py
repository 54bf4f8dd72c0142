"""MI355X (gfx950) library for the bivariate parsimonious-Matern Gaussian
log-likelihood (arxiv 2008.07437): covariance generation, tiled Cholesky,
log-determinant and solve, TLR and mixed-precision variants, cokriging.

The compute path is the HIP library ``libmvgeo.so`` (C ABI in
``include/mvgeo.h``); this package only marshals torch tensors (device memory
and the current stream) into those calls.  There is no CPU fallback: without
the built library or a GPU every call raises.
"""
from ._lib import (  # noqa: F401
    MVG_FP64, MVG_MIXED_FP32, MVG_MIXED_BF16, MVG_TLR, MVG_DST, MVG_MIXED_FP32X,
    MVG_MIXED_BF16X3,
    Opts, Theta, ThetaP, Mat, Factor, MvgError, cov_generate_p, loglik_p, profile_loglik_p,
    mle_fit, MleOpts,
    library_path, morton_order, cov_generate, potrf_tiled, loglik, loglik_many,
    loglik_many_noalloc, tlr_compress,
    cokrige_predict, mloe_mmom, mvg_footprint, mvg_mat_loglik, mvg_dst_band, mvg_autotune_nb, MVG_NB_AUTO, mvg_trmv, mvg_prof_enable, mvg_prof_read, mvg_ir_stats,
    Server, Result, REQ_LOGLIK, REQ_COKRIGE,
)
