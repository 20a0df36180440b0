"""Bayesian shear inference on MI355X (gfx950): HIP kernels behind a C ABI.

The compute path is libbsi.so (hand-written HIP); this package only
marshals arguments.  Importing it does not touch the GPU; the first call does,
and fails loudly if the library has not been built.
"""
from ._native import (PROFILE_EXPONENTIAL, PROFILE_GAUSSIAN, LIK_KSPACE, LIK_PIXEL, METRIC_GIVEN,
                      METRIC_FISHER, FORM_BATCHED, FORM_PLAIN, E_BA14, E_TRUNC_GAUSS,
                      STATUS_OUT_OF_SUPPORT, STATUS_NONFINITE, STATUS_DIVERGENT, LIB_PATH)

__all__ = ["PROFILE_EXPONENTIAL", "PROFILE_GAUSSIAN", "LIK_KSPACE", "LIK_PIXEL", "METRIC_GIVEN",
           "METRIC_FISHER", "FORM_BATCHED", "FORM_PLAIN", "E_BA14", "E_TRUNC_GAUSS",
           "STATUS_OUT_OF_SUPPORT", "STATUS_NONFINITE", "STATUS_DIVERGENT", "LIB_PATH"]
