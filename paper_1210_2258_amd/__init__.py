"""MI355X-native SGP / Richardson-Lucy Poisson deconvolution.

Python face of libsgpdeconv.so (C ABI in include/sgpdeconv.h).  Implements
Prato et al., "Efficient deconvolution methods for astronomical imaging:
algorithms and IDL-GPU codes" (2012): scaled gradient projection with RL
scaling for the Kullback-Leibler divergence, single / multiple images and
boundary-effect correction, plus the RL iterations.
"""
from ._lib import (  # noqa: F401
    EXPORTS, LIB_PATH, REASONS, STOP_CONV, STOP_DISCREPANCY, STOP_FIXED, STOP_RMSE, INIT_DATA, INIT_FLAT,
    INIT_USER, INIT_ZERO, SgpError, apply_operator, default_params, load, release_cache,
    rl_boundary_deconv, rl_deconv, rl_multi_deconv, sgp_boundary_deconv, sgp_deconv,
    sgp_multi_deconv, Solver, steplength_rule, KIND_RL, KIND_SGP, KCLASSES, batch_deconv, INIT_WARM, CnnNet, KIND_OSEM,
    osem_deconv, osem_boundary_deconv, mosaic_deconv, tile_info, set_tile_schedule, get_tile_schedule,
    save_tile_schedule, load_tile_schedule, autotune, flux_multiplier, sgp_deconv_noalloc,
)
