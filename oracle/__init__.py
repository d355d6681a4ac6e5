"""FP64 CPU oracle for asymmetric plmDCA (arXiv:1401.4832), for testing only.

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's CPU
baseline use this package.  The GPU library never imports, links or calls it,
and it shares no code with the GPU library.  The arithmetic lives in
``plm_oracle.c`` (plain loops in FP64); this module only marshals numpy arrays.

Layouts: msa uint8[B, N]; h float64[N, q]; J float64[N, N, q, q] with
J[r, i, k, s] = J^{(r)}_{ri}(s, k) (s = state of site r, k = state of site i).
Objective scale: f_r = B_eff * g_r^reg.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libplm_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle (portable x86-64, IEEE semantics: no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c99", "-ffp-contract=off",
                               "-fno-fast-math", "-o", tmp, os.path.join(_HERE, "plm_oracle.c"),
                               "-lm", "-lpthread"])
        os.replace(tmp, _SO)
    return _SO


class FitOpts(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("c1", ctypes.c_double), ("c2", ctypes.c_double)]


class FitStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("evaluations", ctypes.c_int), ("status", ctypes.c_int),
                ("f", ctypes.c_double), ("gnorm", ctypes.c_double)]


_L = None


def _lib():
    global _L
    if _L is None:
        build(force=not os.path.exists(_SO))
        L = ctypes.CDLL(_SO)
        P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        L.oracle_reweight.argtypes = [P, I, I, D, I, P, P, P, I]
        L.oracle_reweight.restype = None
        L.oracle_reweight_rows.argtypes = [P, I, I, D, P, I, P, I]
        L.oracle_reweight_rows.restype = None
        L.oracle_site_objgrad.argtypes = [P, I, I, I, I, P, D, P, P, D, D, P, P]
        L.oracle_site_objgrad.restype = D
        L.oracle_objgrad.argtypes = [P, I, I, I, P, D, P, P, D, D, P, I, P, P, P, I]
        L.oracle_objgrad.restype = None
        L.oracle_objgrad_slices.argtypes = [P, I, I, I, P, D, P, P, D, D, P, I, P, P, P, I]
        L.oracle_objgrad_slices.restype = None
        L.oracle_site_fit.argtypes = [P, I, I, I, I, P, D, D, D, ctypes.POINTER(FitOpts), P, P,
                                      ctypes.POINTER(FitStats)]
        L.oracle_site_fit.restype = I
        L.oracle_fit.argtypes = [P, I, I, I, P, D, D, D, ctypes.POINTER(FitOpts), P, I, P, P,
                                 ctypes.POINTER(FitStats), I]
        L.oracle_fit.restype = None
        L.oracle_score.argtypes = [P, I, I, P, P]
        L.oracle_score.restype = None
        L.oracle_score_f32.argtypes = [P, I, I, P, P]
        L.oracle_score_f32.restype = None
        _L = L
    return _L


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _threads(n=None):
    if n:
        return n
    try:
        c = len(os.sched_getaffinity(0))
    except Exception:  # pragma: no cover
        c = os.cpu_count() or 1
    return max(1, min(16, c))


def _msa(msa):
    msa = np.ascontiguousarray(msa, dtype=np.uint8)
    assert msa.ndim == 2
    return msa


def reweight(msa, theta=0.8, uniform=False, nthreads=None):
    """(m int32[B], w float64[B], B_eff float) per sec. 3.1 / sec. 3.4 step 2."""
    msa = _msa(msa)
    B, N = msa.shape
    m = np.zeros(B, dtype=np.int32)
    w = np.zeros(B, dtype=np.float64)
    beff = ctypes.c_double(0.0)
    _lib().oracle_reweight(_p(msa), B, N, float(theta), int(bool(uniform)), _p(m), _p(w),
                           ctypes.byref(beff), _threads(nthreads))
    return m, w, beff.value


def reweight_rows(msa, rows, theta=0.8, nthreads=None):
    """m_b for the listed rows only."""
    msa = _msa(msa)
    B, N = msa.shape
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    m = np.zeros(rows.shape[0], dtype=np.int32)
    _lib().oracle_reweight_rows(_p(msa), B, N, float(theta), _p(rows), rows.shape[0], _p(m),
                                _threads(nthreads))
    return m


def site_objgrad(msa, r, w, beff, hr, Jr, lambda_h=0.01, lambda_J=0.01, grad=True):
    """f_r and (gh_r [q], gJ_r [N, q, q]) for one site from its own slices."""
    msa = _msa(msa)
    B, N = msa.shape
    hr = np.ascontiguousarray(hr, dtype=np.float64)
    q = hr.shape[0]
    Jr = np.ascontiguousarray(Jr, dtype=np.float64).reshape(N, q, q)
    w = np.ascontiguousarray(w, dtype=np.float64)
    gh = np.zeros(q) if grad else None
    gJ = np.zeros((N, q, q)) if grad else None
    f = _lib().oracle_site_objgrad(_p(msa), B, N, q, int(r), _p(w), float(beff), _p(hr), _p(Jr),
                                   float(lambda_h), float(lambda_J),
                                   _p(gh) if grad else None, _p(gJ) if grad else None)
    return (f, gh, gJ) if grad else f


def objgrad(msa, w, beff, h, J, lambda_h=0.01, lambda_J=0.01, sites=None, nthreads=None):
    """Per-site f [ns], gh [ns, q], gJ [ns, N, q, q] for the listed sites."""
    msa = _msa(msa)
    B, N = msa.shape
    h = np.ascontiguousarray(h, dtype=np.float64)
    q = h.shape[1]
    J = np.ascontiguousarray(J, dtype=np.float64).reshape(N, N, q, q)
    w = np.ascontiguousarray(w, dtype=np.float64)
    sites = np.arange(N, dtype=np.int32) if sites is None else np.ascontiguousarray(sites, dtype=np.int32)
    ns = sites.shape[0]
    f = np.zeros(ns)
    gh = np.zeros((ns, q))
    gJ = np.zeros((ns, N, q, q))
    _lib().oracle_objgrad(_p(msa), B, N, q, _p(w), float(beff), _p(h), _p(J), float(lambda_h),
                          float(lambda_J), _p(sites), ns, _p(f), _p(gh), _p(gJ), _threads(nthreads))
    return f, gh, gJ


def objgrad_slices(msa, w, beff, hr, Jr, sites, lambda_h=0.01, lambda_J=0.01, grad=True,
                   nthreads=None):
    """objgrad for the listed sites from their own slices hr [ns, q], Jr [ns, N, q, q]."""
    msa = _msa(msa)
    B, N = msa.shape
    sites = np.ascontiguousarray(sites, dtype=np.int32)
    ns = sites.shape[0]
    hr = np.ascontiguousarray(hr, dtype=np.float64).reshape(ns, -1)
    q = hr.shape[1]
    Jr = np.ascontiguousarray(Jr, dtype=np.float64).reshape(ns, N, q, q)
    w = np.ascontiguousarray(w, dtype=np.float64)
    f = np.zeros(ns)
    gh = np.zeros((ns, q)) if grad else None
    gJ = np.zeros((ns, N, q, q)) if grad else None
    _lib().oracle_objgrad_slices(_p(msa), B, N, q, _p(w), float(beff), _p(hr), _p(Jr),
                                 float(lambda_h), float(lambda_J), _p(sites), ns, _p(f),
                                 _p(gh) if grad else None, _p(gJ) if grad else None,
                                 _threads(nthreads))
    return f, gh, gJ


def fit(msa, w, beff, lambda_h=0.01, lambda_J=0.01, sites=None, q=21, tol=1e-8, max_iter=10000,
        m=10, c1=1e-4, c2=0.9, nthreads=None):
    """Per-site minimisers from zero: h [ns, q], J [ns, N, q, q], stats list."""
    msa = _msa(msa)
    B, N = msa.shape
    w = np.ascontiguousarray(w, dtype=np.float64)
    sites = np.arange(N, dtype=np.int32) if sites is None else np.ascontiguousarray(sites, dtype=np.int32)
    ns = sites.shape[0]
    h = np.zeros((ns, q))
    J = np.zeros((ns, N, q, q))
    st = (FitStats * ns)()
    opts = FitOpts(m, tol, max_iter, c1, c2)
    _lib().oracle_fit(_p(msa), B, N, q, _p(w), float(beff), float(lambda_h), float(lambda_J),
                      ctypes.byref(opts), _p(sites), ns, _p(h), _p(J), st, _threads(nthreads))
    stats = [dict(iterations=s.iterations, evaluations=s.evaluations, status=s.status, f=s.f,
                  gnorm=s.gnorm) for s in st]
    return h, J, stats


def score(J):
    """(FN, CFN) float64 [N, N] from J [N, N, q, q] (float32 or float64)."""
    J = np.asarray(J)
    N, _, q, _ = J.shape
    fn = np.zeros((N, N))
    cfn = np.zeros((N, N))
    if J.dtype == np.float32:
        J = np.ascontiguousarray(J)
        _lib().oracle_score_f32(_p(J), N, q, _p(fn), _p(cfn))
    else:
        J = np.ascontiguousarray(J, dtype=np.float64)
        _lib().oracle_score(_p(J), N, q, _p(fn), _p(cfn))
    return fn, cfn
