"""MI355X FFT-CONV for truncated matrix power series and the TEK NSPT step.

The computation lives in libpolymat.so (hand-written HIP kernels for gfx950
behind the C ABI of include/polymat.h); this package is its Python binding.
"""
from ._native import (PM_OK, PM_ERR_INVALID, PM_ERR_WORKSPACE, PM_ERR_DEVICE, PM_ERR_UNSUPPORTED,
                      PM_ERR_NONFINITE,
                      PM_PREC_FP64, PM_PREC_FP32, PM_PREC_BF16X3, PM_OP_N, PM_OP_C, PolymatError,
                      LIB_PATH, NOALLOC_SCRATCH_BYTES, lib)
from .api import (polymat_mul, polymat_mul_noalloc, polymat_mul_naive, polymat_mul_batched, batched_workspace_size, workspace_size,
                  forward_transform, inverse_transform, transform_length, nspt_params,
                  nspt_workspace_size, nspt_langevin_step, nspt_langevin_steps, nspt_noise, nspt_md_trajectory,
                  nspt_gauge_fix, nspt_action,
                  nspt_wilson_loop,
                  workspace, check_enable, timing_enable,
                  timing_read)

__all__ = [
    "polymat_mul", "polymat_mul_noalloc", "polymat_mul_naive", "polymat_mul_batched", "batched_workspace_size", "workspace_size",
    "forward_transform", "inverse_transform", "transform_length", "nspt_params",
    "nspt_workspace_size", "nspt_langevin_step", "nspt_langevin_steps", "nspt_noise", "nspt_md_trajectory",
    "nspt_gauge_fix", "nspt_action", "nspt_wilson_loop", "workspace", "check_enable", "timing_enable", "timing_read", "lib", "LIB_PATH", "PolymatError",
]
