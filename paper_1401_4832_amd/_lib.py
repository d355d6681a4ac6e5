"""ctypes declarations of libplm's C ABI (include/plm.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libplm.so")

PLM_OK = 0
PLM_W_MAXITER = 1
PLM_E_INVALID = -1
PLM_E_SYMBOL = -2
PLM_E_NONFINITE = -3
PLM_E_WORKSPACE = -4
PLM_E_HIP = -5
PLM_E_UNSUPPORTED = -6

PATH_GATHER_FP32 = 0
PATH_MFMA_BF16X2 = 1
PATH_GATHER_MFMA_FP32 = 2
PATH_MFMA_FP32 = 3
PATH_GATHER_MFMA_F16X2 = 4
PATH_GATHER_MFMA_I8X3 = 5
PATH_MFMA_I8X3 = 6
PATH_GATHER64_MFMA_I8X6 = 7

STATIC_SCRATCH_BYTES = 64 << 20

SITE_STATUS = {0: "converged", 1: "maxiter", 2: "linesearch", 3: "nonfinite"}


class FitOpts(ctypes.Structure):
    _fields_ = [
        ("lambda_h", ctypes.c_double),
        ("lambda_J", ctypes.c_double),
        ("tol", ctypes.c_double),
        ("max_iter", ctypes.c_int32),
        ("lbfgs_m", ctypes.c_int32),
        ("max_linesearch", ctypes.c_int32),
        ("path", ctypes.c_int32),
        ("sync_every", ctypes.c_int32),
        ("use_graph", ctypes.c_int32),
        ("single_site", ctypes.c_int32),
        ("tile_seqs", ctypes.c_int32),
        ("site_limit", ctypes.c_int32),
        ("timing", ctypes.c_int32),
        ("refine", ctypes.c_int32),
        ("n_probe", ctypes.c_int32),
        ("refine_tol", ctypes.c_double),
        ("probe_sites", ctypes.c_void_p),
        ("probe_h", ctypes.c_void_p),
        ("probe_J", ctypes.c_void_p),
        ("probe_out", ctypes.c_void_p),
        ("probe_count", ctypes.c_void_p),
        ("probe_cap", ctypes.c_int32),
        ("history_fp64", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 2),
    ]


class FitTiming(ctypes.Structure):
    _fields_ = [
        ("forward_ms", ctypes.c_double),
        ("backward_ms", ctypes.c_double),
        ("lbfgs_ms", ctypes.c_double),
        ("total_ms", ctypes.c_double),
        ("iterations", ctypes.c_int64),
        ("site_evals", ctypes.c_int64),
        ("quant_ms", ctypes.c_double),
        ("refine_forward_ms", ctypes.c_double),
        ("refine_backward_ms", ctypes.c_double),
        ("refine_lbfgs_ms", ctypes.c_double),
        ("refine_iterations", ctypes.c_int64),
        ("refine_site_evals", ctypes.c_int64),
    ]


class SiteStats(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int32),
        ("evaluations", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("pad", ctypes.c_int32),
        ("f", ctypes.c_double),
        ("gnorm", ctypes.c_double),
    ]


class MsaDesc(ctypes.Structure):
    _fields_ = [
        ("msa", ctypes.c_void_p),
        ("B", ctypes.c_int32),
        ("N", ctypes.c_int32),
        ("w", ctypes.c_void_p),
        ("beff", ctypes.c_void_p),
        ("h_io", ctypes.c_void_p),
        ("J_io", ctypes.c_void_p),
        ("stats_out", ctypes.POINTER(SiteStats)),
    ]


class TuneResult(ctypes.Structure):
    _fields_ = [
        ("path", ctypes.c_int32),
        ("tile_seqs", ctypes.c_int32),
        ("eval_ms", ctypes.c_double),
    ]


class ScoreOpts(ctypes.Structure):
    _fields_ = [
        ("combine", ctypes.c_int32),
        ("norm", ctypes.c_int32),
        ("p", ctypes.c_double),
        ("exclude_gap", ctypes.c_int32),
        ("correction", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 4),
    ]


FORMAT = {"auto": 0, "fasta": 1, "stockholm": 2}
COMBINE = {"avg": 0, "min": 1, "max": 2}
NORM = {"frob": 0, "lp": 1, "burkoff": 2}
CORRECTION = {"apc": 0, "none": 1, "asc": 2}


class PlmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libplm status {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libplm.so; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "or python -m paper_1401_4832_amd._build")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, D, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
        sig = {
            "plm_ctx_create": (ctypes.c_int, [ctypes.POINTER(P), ctypes.c_int, P]),
            "plm_ctx_destroy": (ctypes.c_int, [P]),
            "plm_last_error": (ctypes.c_char_p, [P]),
            "plm_status_string": (ctypes.c_char_p, [ctypes.c_int]),
            "plm_sync": (ctypes.c_int, [P]),
            "plm_reweight": (ctypes.c_int, [P, P, I32, I32, I32, D, I32, P, P, P]),
            "plm_objgrad_workspace_bytes": (SZ, [I32, I32, I32, I32]),
            "plm_objgrad": (ctypes.c_int, [P, P, I32, I32, I32, P, P, P, P, D, D, P, I32, I32, P, SZ,
                                           P, P, P, P]),
            "plm_objgrad_static": (ctypes.c_int, [P, P, I32, I32, I32, P, P, P, P, D, D, P, I32, I32, P, P, P, P]),
            "plm_fit_opts_default": (None, [ctypes.POINTER(FitOpts)]),
            "plm_fit_opts_size": (SZ, []),
            "plm_fit_workspace_bytes": (SZ, [I32, I32, I32, ctypes.POINTER(FitOpts)]),
            "plm_fit": (ctypes.c_int, [P, P, I32, I32, I32, P, P, ctypes.POINTER(FitOpts), P, SZ, P, P,
                                       ctypes.POINTER(SiteStats)]),
            "plm_score": (ctypes.c_int, [P, P, I32, I32, P, P]),
            "plm_fit_last_timing": (ctypes.c_int, [P, ctypes.POINTER(FitTiming)]),
            "plm_fit_batch_workspace_bytes": (SZ, [ctypes.POINTER(MsaDesc), I32, I32, ctypes.POINTER(FitOpts)]),
            "plm_fit_batch": (ctypes.c_int, [P, ctypes.POINTER(MsaDesc), I32, I32, ctypes.POINTER(FitOpts),
                                             P, SZ]),
            "plm_score_opts_default": (None, [ctypes.POINTER(ScoreOpts)]),
            "plm_frequencies": (ctypes.c_int, [P, P, I32, I32, I32, P, P, P]),
            "plm_score_ex": (ctypes.c_int, [P, P, I32, I32, ctypes.POINTER(ScoreOpts), P, P, P]),
            "plm_contact_tpr": (ctypes.c_int, [P, P, I32, P, I32, I32, P, ctypes.POINTER(I32)]),
            "plm_parse_alignment": (ctypes.c_int, [ctypes.c_char_p, SZ, I32, P, SZ, ctypes.POINTER(I32),
                                                   ctypes.POINTER(I32), ctypes.c_char_p, SZ]),
            "plm_fit_symmetric_workspace_bytes": (SZ, [I32, I32, I32, ctypes.POINTER(FitOpts)]),
            "plm_fit_symmetric": (ctypes.c_int, [P, P, I32, I32, I32, P, P, ctypes.POINTER(FitOpts), P, SZ, P,
                                                 P, ctypes.POINTER(SiteStats)]),
            "plm_fit_symmetric_split": (ctypes.c_int, [P, P, I32, I32, I32, P, P, ctypes.POINTER(FitOpts), P, SZ,
                                                       P, P, P, P, ctypes.POINTER(SiteStats)]),
            "plm_mf_init_workspace_bytes": (SZ, [I32, I32, I32]),
            "plm_mf_init": (ctypes.c_int, [P, P, I32, I32, I32, P, P, D, P, SZ, P, P]),
            "plm_tune": (ctypes.c_int, [P, ctypes.POINTER(MsaDesc), I32, I32, ctypes.POINTER(FitOpts), I32, P,
                                        SZ, ctypes.POINTER(TuneResult), I32, ctypes.POINTER(I32)]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    """Names declared in include/plm.h that the ABI tests check for."""
    return ["plm_ctx_create", "plm_ctx_destroy", "plm_last_error", "plm_status_string", "plm_sync",
            "plm_reweight", "plm_objgrad_workspace_bytes", "plm_objgrad", "plm_fit_opts_default",
            "plm_fit_opts_size", "plm_objgrad_static",
            "plm_fit_workspace_bytes", "plm_fit", "plm_score", "plm_fit_last_timing",
            "plm_fit_batch_workspace_bytes", "plm_fit_batch", "plm_tune", "plm_score_opts_default",
            "plm_frequencies", "plm_score_ex", "plm_contact_tpr", "plm_parse_alignment",
            "plm_fit_symmetric_workspace_bytes", "plm_fit_symmetric", "plm_fit_symmetric_split",
            "plm_mf_init_workspace_bytes", "plm_mf_init"]
