"""MI355X (gfx950) asymmetric plmDCA: pseudolikelihood objective, gradient,
batched L-BFGS fit and coupling scores behind the C ABI of include/plm.h.

Method: Ekeberg, Hartonen & Aurell, arXiv:1401.4832 (sec. 3.4 rundown)."""
from . import _lib
from .autograd import PLMObjective, plm_objective
from . import autotune
from .api import (FitOptions, FitResult, Probe, contact_tpr, context, fit, fit_batch, fit_symmetric, frequencies, mf_init, last_fit_timing,
                  objgrad, objgrad_static, parse_alignment, read_alignment, reweight, score, sync, tune, workspace)
from ._lib import (PATH_GATHER_FP32, PATH_GATHER_MFMA_F16X2, PATH_GATHER_MFMA_FP32, PATH_GATHER_MFMA_I8X3,
                   PATH_MFMA_BF16X2,
                   PATH_MFMA_FP32, PATH_MFMA_I8X3, PATH_GATHER64_MFMA_I8X6, PlmError)

__all__ = ["PLMObjective", "plm_objective", "FitOptions", "FitResult", "context", "fit", "fit_batch", "fit_symmetric", "mf_init",
           "last_fit_timing", "objgrad", "reweight", "score", "sync", "tune", "autotune", "workspace",
           "frequencies", "contact_tpr", "parse_alignment", "read_alignment", "PATH_GATHER_FP32", "PATH_GATHER_MFMA_FP32", "PATH_MFMA_BF16X2",
           "PATH_MFMA_FP32", "PATH_GATHER_MFMA_F16X2", "PATH_GATHER_MFMA_I8X3", "PATH_MFMA_I8X3", "PlmError"]
