"""MI355X (gfx950) LM bundle-adjustment step of InstantSfM (arXiv 2510.13310).

The computation lives in ``libinstantba.so`` (HIP kernels + native host orchestration behind
the C ABI of ``include/ba.h``); this package is its thin Python binding and the
``torch.autograd.Function`` wrapper of the implicit adjoint.
"""
from ._abi import (BAError, BA_OK, BA_EMPTY, BA_NOT_CONVERGED, BA_ERR_ARG, BA_ERR_STATE, BA_ERR_OOM,
                   BA_ERR_DEVICE, BA_ERR_NUMERIC, BA_PRECISION_FP64, BA_PRECISION_MIXED,
                   LIB_PATH, load)
from .api import (BundleAdjuster, make_options, ba_default_options, ba_create,
                  ba_set_observations, ba_set_depth_priors, ba_set_fixed_cameras, ba_lm_step,
                  ba_lm_step_noalloc, ba_solve, ba_get_params, ba_get_intrinsics, ba_set_params, ba_get_active,
                  ba_get_last_step,
                  ba_get_normal_blocks, ba_get_preconditioner, ba_adjoint, ba_kernel_stats, ba_reset_kernel_stats,
                  ba_device_bytes, ba_last_error, ba_destroy, ba_gp_step, ba_gp_solve,
                  ba_gp_get_scales, ba_gp_reset)

__all__ = [
    "BAError", "BA_OK", "BA_EMPTY", "BA_NOT_CONVERGED", "BA_ERR_ARG", "BA_ERR_STATE", "BA_ERR_OOM",
    "BA_ERR_DEVICE", "BA_ERR_NUMERIC", "BA_PRECISION_FP64", "BA_PRECISION_MIXED", "LIB_PATH",
    "load", "BundleAdjuster", "make_options", "ba_default_options", "ba_create",
    "ba_set_observations", "ba_set_depth_priors", "ba_set_fixed_cameras", "ba_lm_step",
    "ba_lm_step_noalloc", "ba_solve", "ba_get_params", "ba_get_intrinsics", "ba_set_params", "ba_get_active",
    "ba_get_last_step",
    "ba_get_normal_blocks", "ba_get_preconditioner", "ba_adjoint", "ba_kernel_stats", "ba_reset_kernel_stats",
    "ba_device_bytes", "ba_last_error", "ba_destroy", "ba_gp_step", "ba_gp_solve",
    "ba_gp_get_scales", "ba_gp_reset",
]
