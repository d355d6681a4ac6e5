"""Python binding of libplm over torch tensors (device memory and streams only).

Every function marshals tensors into the C ABI of include/plm.h; all arithmetic
runs in the library's HIP kernels on the tensor's device, on the current
stream.  There is no CPU fallback: without the built library or a gfx950
device the calls raise.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import torch

from . import _lib as L

_ctx_cache: dict = {}


def _check(rc: int, ctx) -> int:
    if rc < 0:
        msg = L.lib().plm_last_error(ctx).decode() if ctx else L.lib().plm_status_string(rc).decode()
        raise L.PlmError(rc, msg)
    return rc


def context(device=None):
    """The library context bound to `device` and torch's current stream there."""
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    if dev.type != "cuda":
        raise ValueError("libplm runs on a GPU device")
    idx = dev.index if dev.index is not None else torch.cuda.current_device()
    stream = torch.cuda.current_stream(idx).cuda_stream
    key = (idx, stream)
    c = _ctx_cache.get(key)
    if c is None:
        p = ctypes.c_void_p()
        rc = L.lib().plm_ctx_create(ctypes.byref(p), idx, ctypes.c_void_p(stream))
        if rc != 0:
            raise L.PlmError(rc, L.lib().plm_status_string(rc).decode())
        c = p
        _ctx_cache[key] = c
    return c


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dev_tensor(t, dtype, device, name):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def sync(device=None):
    ctx = context(device)
    _check(L.lib().plm_sync(ctx), ctx)


def reweight(msa: torch.Tensor, theta: float = 0.8, uniform: bool = False, q: int = 21):
    """(m int32[B], w float64[B], beff float64[1]) on msa's device (sec. 3.1)."""
    dev = msa.device
    _dev_tensor(msa, torch.uint8, dev, "msa")
    B, N = msa.shape
    m = torch.empty(B, dtype=torch.int32, device=dev)
    w = torch.empty(B, dtype=torch.float64, device=dev)
    beff = torch.empty(1, dtype=torch.float64, device=dev)
    ctx = context(dev)
    _check(L.lib().plm_reweight(ctx, _ptr(msa), B, N, q, float(theta), int(bool(uniform)), _ptr(m),
                                _ptr(w), _ptr(beff)), ctx)
    return m, w, beff


def objgrad(msa, w, beff, h, J, lambda_h=0.01, lambda_J=0.01, sites=None, grad=True,
            path=L.PATH_GATHER_FP32, grad_scale=None):
    """f float64[N], gh float32[N,q], gJ float32[N,N,q,q] for the listed sites (all if None).

    Rows of unlisted sites are left zero.  f_r = B_eff * g_r^reg.  With
    grad_scale (float64 [N] on the device) the gradient rows of site r are
    multiplied by grad_scale[r] inside the library."""
    dev = msa.device
    _dev_tensor(msa, torch.uint8, dev, "msa")
    B, N = msa.shape
    q = h.shape[1]
    _dev_tensor(w, torch.float64, dev, "w")
    _dev_tensor(beff, torch.float64, dev, "beff")
    _dev_tensor(h, torch.float32, dev, "h")
    _dev_tensor(J, torch.float32, dev, "J")
    if tuple(J.shape) != (N, N, q, q) or tuple(h.shape) != (N, q) or w.numel() != B:
        raise ValueError("shape mismatch between msa, w, h and J")
    if sites is not None:
        sites = torch.as_tensor(sites, dtype=torch.int32).to(dev).contiguous()
        ns = int(sites.numel())
    else:
        ns = N
    if grad_scale is not None:
        _dev_tensor(grad_scale, torch.float64, dev, "grad_scale")
        if grad_scale.numel() != N:
            raise ValueError("grad_scale must have N entries")
    f = torch.zeros(N, dtype=torch.float64, device=dev)
    gh = torch.zeros(N, q, dtype=torch.float32, device=dev) if grad else None
    gJ = torch.zeros(N, N, q, q, dtype=torch.float32, device=dev) if grad else None
    nbytes = L.lib().plm_objgrad_workspace_bytes(B, N, q, path)
    ws = workspace(nbytes, dev)
    ctx = context(dev)
    _check(L.lib().plm_objgrad(ctx, _ptr(msa), B, N, q, _ptr(w), _ptr(beff), _ptr(h), _ptr(J),
                               float(lambda_h), float(lambda_J), _ptr(sites), ns, path, _ptr(ws),
                               ws.numel(), _ptr(grad_scale), _ptr(f), _ptr(gh), _ptr(gJ)), ctx)
    return f, gh, gJ


def objgrad_static(msa, w, beff, h, J, lambda_h=0.01, lambda_J=0.01, sites=None, grad=True,
                   path=L.PATH_GATHER_FP32, grad_scale=None, out=None):
    """objgrad() through plm_objgrad_static: no workspace, the library's fixed
    scratch array (problems up to L.STATIC_SCRATCH_BYTES of scratch).  out may
    hold preallocated (f, gh, gJ) tensors, so that the call allocates nothing."""
    dev = msa.device
    _dev_tensor(msa, torch.uint8, dev, "msa")
    B, N = msa.shape
    q = h.shape[1]
    _dev_tensor(w, torch.float64, dev, "w")
    _dev_tensor(beff, torch.float64, dev, "beff")
    _dev_tensor(h, torch.float32, dev, "h")
    _dev_tensor(J, torch.float32, dev, "J")
    if tuple(J.shape) != (N, N, q, q) or tuple(h.shape) != (N, q) or w.numel() != B:
        raise ValueError("shape mismatch between msa, w, h and J")
    if sites is not None:
        sites = _dev_tensor(sites, torch.int32, dev, "sites") if isinstance(sites, torch.Tensor) else \
            torch.as_tensor(sites, dtype=torch.int32).to(dev).contiguous()
        ns = int(sites.numel())
    else:
        ns = N
    if grad_scale is not None:
        _dev_tensor(grad_scale, torch.float64, dev, "grad_scale")
    if out is None:
        f = torch.zeros(N, dtype=torch.float64, device=dev)
        gh = torch.zeros(N, q, dtype=torch.float32, device=dev) if grad else None
        gJ = torch.zeros(N, N, q, q, dtype=torch.float32, device=dev) if grad else None
    else:
        f, gh, gJ = out
    ctx = context(dev)
    _check(L.lib().plm_objgrad_static(ctx, _ptr(msa), B, N, q, _ptr(w), _ptr(beff), _ptr(h), _ptr(J),
                                      float(lambda_h), float(lambda_J), _ptr(sites), ns, path,
                                      _ptr(grad_scale), _ptr(f), _ptr(gh), _ptr(gJ)), ctx)
    return f, gh, gJ


@dataclass
class FitOptions:
    lambda_h: float = 0.01
    lambda_J: float = 0.01
    tol: float = 1e-6
    max_iter: int = 2000
    lbfgs_m: int = 10
    max_linesearch: int = 20
    path: int = L.PATH_GATHER_FP32
    sync_every: int = 8
    use_graph: bool = True
    single_site: bool = False
    tile_seqs: int = 0
    site_limit: int = 0
    timing: bool = False
    # a second fit from the first one's point on another path: 0 automatic
    # (path 6 is refined on path 5, path 1 on path 3), -1 never, 1 + p always on path p
    refine: int = 0
    # pick path and tile_seqs with the autotuner (cached per size bucket)
    autotune: bool = False
    # tolerance of the refinement fit (0: tol)
    refine_tol: float = 0.0
    # curvature pairs and the gradient kept at the iterate in FP64 (default FP32)
    history_fp64: bool = False

    def to_c(self) -> L.FitOpts:
        o = L.FitOpts()
        L.lib().plm_fit_opts_default(ctypes.byref(o))
        for k in ("lambda_h", "lambda_J", "tol", "refine_tol"):
            setattr(o, k, float(getattr(self, k)))
        for k in ("max_iter", "lbfgs_m", "max_linesearch", "path", "sync_every", "tile_seqs", "site_limit",
                  "refine"):
            setattr(o, k, int(getattr(self, k)))
        o.use_graph = int(bool(self.use_graph))
        o.single_site = int(bool(self.single_site))
        o.timing = int(bool(self.timing))
        o.history_fp64 = int(bool(self.history_fp64))
        return o


@dataclass
class Probe:
    """Convergence probe of fit(): after the start point and after every
    iteration, the device records its wall clock (seconds) and the max-abs
    difference between the iterate and reference values (h_ref [n, q],
    J_ref [n, N, q, q], float32 on the device) for the watched sites."""
    sites: torch.Tensor
    h_ref: torch.Tensor
    J_ref: torch.Tensor
    cap: int = 20000


@dataclass
class FitResult:
    h: torch.Tensor
    J: torch.Tensor
    stats: list = field(default_factory=list)
    status: int = 0
    # probe entries (numpy [count, 2 + n]: time s, max over sites, per site), if probed
    probe: object = None
    # low-order words of the parameters (fit_symmetric(..., split=True)): the
    # point is h + h_lo, J + J_lo, each pair summed in FP64
    h_lo: object = None
    J_lo: object = None

    @property
    def evaluations(self) -> int:
        return int(sum(s["evaluations"] for s in self.stats))


def fit(msa, w, beff, opts: FitOptions | None = None, h0=None, J0=None, probe: Probe | None = None) -> FitResult:
    """Minimise every site's g_r^reg (sec. 3.4 step 3) from (h0, J0) (zeros by default)."""
    opts = opts or FitOptions()
    if opts.autotune and not opts.single_site:
        from . import autotune
        opts = autotune.tuned_options([(msa, w, beff)], opts, 21 if h0 is None else h0.shape[1])
    dev = msa.device
    _dev_tensor(msa, torch.uint8, dev, "msa")
    B, N = msa.shape
    q = 21 if h0 is None else h0.shape[1]
    h = torch.zeros(N, q, dtype=torch.float32, device=dev) if h0 is None else h0.clone().contiguous()
    J = torch.zeros(N, N, q, q, dtype=torch.float32, device=dev) if J0 is None else J0.clone().contiguous()
    _dev_tensor(w, torch.float64, dev, "w")
    _dev_tensor(beff, torch.float64, dev, "beff")
    co = opts.to_c()
    pout = pcount = None
    if probe is not None:
        sites = _dev_tensor(probe.sites, torch.int32, dev, "probe.sites")
        n = int(sites.numel())
        _dev_tensor(probe.h_ref, torch.float32, dev, "probe.h_ref")
        _dev_tensor(probe.J_ref, torch.float32, dev, "probe.J_ref")
        if tuple(probe.h_ref.shape) != (n, q) or tuple(probe.J_ref.shape) != (n, N, q, q):
            raise ValueError("probe reference shapes must be [n, q] and [n, N, q, q]")
        pout = torch.full((int(probe.cap), 2 + n), float("nan"), dtype=torch.float64, device=dev)
        pcount = torch.zeros(1, dtype=torch.int32, device=dev)
        co.n_probe = n
        co.probe_sites, co.probe_h, co.probe_J = sites.data_ptr(), probe.h_ref.data_ptr(), probe.J_ref.data_ptr()
        co.probe_out, co.probe_count, co.probe_cap = pout.data_ptr(), pcount.data_ptr(), int(probe.cap)
    nbytes = L.lib().plm_fit_workspace_bytes(B, N, q, ctypes.byref(co))
    if nbytes == 0:
        raise L.PlmError(L.PLM_E_INVALID, "invalid sizes or options")
    ws = workspace(nbytes, dev)
    stats = (L.SiteStats * N)()
    ctx = context(dev)
    rc = _check(L.lib().plm_fit(ctx, _ptr(msa), B, N, q, _ptr(w), _ptr(beff), ctypes.byref(co), _ptr(ws),
                                ws.numel(), _ptr(h), _ptr(J), stats), ctx)
    del ws
    entries = None
    if probe is not None:
        cnt = int(pcount.item())
        entries = pout[:cnt].cpu().numpy()
    return FitResult(h, J, _stats_list(stats), rc, entries)


def fit_symmetric(msa, w, beff, opts: FitOptions | None = None, h0=None, J0=None, split: bool = False,
                  h0_lo=None, J0_lo=None) -> FitResult:
    """Symmetric pseudolikelihood maximisation (sec. 3.2, eqs. npll_1 / l2reg):
    one minimisation of sum_r g_r + lambda_h sum ||h||^2 + lambda_J sum_{i<j} ||J_ij||^2
    with every J_ij shared by sites i and j.  The start point takes the blocks
    J0[r][i], r < i (zeros by default); the result holds J[i][r] = J[r][i]
    with the state axes swapped.  stats holds one record for the whole problem.
    split=True carries every parameter as two FP32 words (plm_fit_symmetric_split;
    start low words h0_lo, J0_lo, zeros by default): the result's h_lo, J_lo
    hold the low words."""
    opts = opts or FitOptions()
    dev = msa.device
    _dev_tensor(msa, torch.uint8, dev, "msa")
    B, N = msa.shape
    q = 21 if h0 is None else h0.shape[1]
    if opts.autotune:
        # the tolerance bounds the gradient norm over all N(N-1)/2 q^2 + N q
        # parameters: the int8 gradient is a candidate only where its rounding
        # noise summed over that many entries stays below half the tolerance
        # (its fit is then refined on an FP32-class path by the library)
        from . import autotune
        opts = autotune.tuned_options([(msa, w, beff)], opts, q, symmetric=True)
    h = torch.zeros(N, q, dtype=torch.float32, device=dev) if h0 is None else h0.clone().contiguous()
    J = torch.zeros(N, N, q, q, dtype=torch.float32, device=dev) if J0 is None else J0.clone().contiguous()
    _dev_tensor(w, torch.float64, dev, "w")
    _dev_tensor(beff, torch.float64, dev, "beff")
    co = opts.to_c()
    nbytes = L.lib().plm_fit_symmetric_workspace_bytes(B, N, q, ctypes.byref(co))
    if nbytes == 0:
        raise L.PlmError(L.PLM_E_INVALID, "invalid sizes or options")
    ws = workspace(nbytes, dev)
    stats = (L.SiteStats * 1)()
    ctx = context(dev)
    if not split:
        if h0_lo is not None or J0_lo is not None:
            raise ValueError("start low words need split=True")
        rc = _check(L.lib().plm_fit_symmetric(ctx, _ptr(msa), B, N, q, _ptr(w), _ptr(beff), ctypes.byref(co),
                                              _ptr(ws), ws.numel(), _ptr(h), _ptr(J), stats), ctx)
        del ws
        return FitResult(h, J, _stats_list(stats), rc)
    hl = torch.zeros_like(h) if h0_lo is None else h0_lo.clone().contiguous()
    Jl = torch.zeros_like(J) if J0_lo is None else J0_lo.clone().contiguous()
    _dev_tensor(hl, torch.float32, dev, "h0_lo")
    _dev_tensor(Jl, torch.float32, dev, "J0_lo")
    if hl.shape != h.shape or Jl.shape != J.shape:
        raise ValueError("low-order words must have the shapes of h and J")
    rc = _check(L.lib().plm_fit_symmetric_split(ctx, _ptr(msa), B, N, q, _ptr(w), _ptr(beff), ctypes.byref(co),
                                                _ptr(ws), ws.numel(), _ptr(h), _ptr(J), _ptr(hl), _ptr(Jl),
                                                stats), ctx)
    del ws
    return FitResult(h, J, _stats_list(stats), rc, h_lo=hl, J_lo=Jl)


def mf_init(msa, w, beff, pseudocount: float = 0.5, q: int = 21):
    """Mean-field starting guess (h [N, q], J [N, N, q, q] float32): couplings
    from the inverse of the pseudocount-regularised connected correlation
    matrix (sec. 2), gap as reference state, in the layout of fit(); pass them
    as fit(..., h0=h, J0=J)."""
    dev = msa.device
    _dev_tensor(msa, torch.uint8, dev, "msa")
    _dev_tensor(w, torch.float64, dev, "w")
    _dev_tensor(beff, torch.float64, dev, "beff")
    B, N = msa.shape
    nbytes = L.lib().plm_mf_init_workspace_bytes(B, N, q)
    if nbytes == 0:
        raise L.PlmError(L.PLM_E_INVALID, "invalid sizes")
    h = torch.empty(N, q, dtype=torch.float32, device=dev)
    J = torch.empty(N, N, q, q, dtype=torch.float32, device=dev)
    ws = workspace(nbytes, dev)
    ctx = context(dev)
    _check(L.lib().plm_mf_init(ctx, _ptr(msa), B, N, q, _ptr(w), _ptr(beff), float(pseudocount), _ptr(ws),
                               ws.numel(), _ptr(h), _ptr(J)), ctx)
    del ws
    return h, J


def _stats_list(stats):
    return [dict(iterations=s.iterations, evaluations=s.evaluations, status=L.SITE_STATUS.get(s.status, "?"),
                 f=s.f, gnorm=s.gnorm) for s in stats]


def _batch_descs(items, q):
    """C descriptors of a batch; returns (descs, [(h, J, stats)])."""
    dev = items[0][0].device
    n = len(items)
    descs = (L.MsaDesc * n)()
    out = []
    for k, it in enumerate(items):
        msa, w, beff = it[0], it[1], it[2]
        _dev_tensor(msa, torch.uint8, dev, f"msa[{k}]")
        _dev_tensor(w, torch.float64, dev, f"w[{k}]")
        _dev_tensor(beff, torch.float64, dev, f"beff[{k}]")
        B, N = msa.shape
        h = torch.zeros(N, q, dtype=torch.float32, device=dev) if len(it) < 4 else it[3].clone().contiguous()
        J = torch.zeros(N, N, q, q, dtype=torch.float32, device=dev) if len(it) < 5 else it[4].clone().contiguous()
        stats = (L.SiteStats * N)()
        d = descs[k]
        d.msa, d.B, d.N, d.w, d.beff = msa.data_ptr(), B, N, w.data_ptr(), beff.data_ptr()
        d.h_io, d.J_io = h.data_ptr(), J.data_ptr()
        d.stats_out = ctypes.cast(stats, ctypes.POINTER(L.SiteStats))
        out.append((h, J, stats))
    return descs, out


def fit_batch(items, opts: FitOptions | None = None, q: int = 21):
    """Fit a ragged batch of alignments in one set of launches per iteration.

    items: sequence of (msa, w, beff) or (msa, w, beff, h0, J0) on one device.
    Returns one FitResult per alignment, in the order given; each equals what
    fit() gives for that alignment alone (with the same tile_seqs)."""
    opts = opts or FitOptions()
    if not items:
        raise ValueError("empty batch")
    if opts.autotune:
        from . import autotune
        opts = autotune.tuned_options(items, opts, q)
    dev = items[0][0].device
    n = len(items)
    descs, out = _batch_descs(items, q)
    co = opts.to_c()
    nbytes = L.lib().plm_fit_batch_workspace_bytes(descs, n, q, ctypes.byref(co))
    if nbytes == 0:
        raise L.PlmError(L.PLM_E_INVALID, "invalid sizes or options")
    ws = workspace(nbytes, dev)
    ctx = context(dev)
    rc = _check(L.lib().plm_fit_batch(ctx, descs, n, q, ctypes.byref(co), _ptr(ws), ws.numel()), ctx)
    del ws
    return [FitResult(h, J, _stats_list(st), rc) for (h, J, st) in out]


def tune(items, opts: FitOptions | None = None, q: int = 21, fp32_only: bool = True) -> list:
    """Time every candidate schedule on the batch (plm_tune); fastest first."""
    opts = opts or FitOptions()
    if not items:
        raise ValueError("empty batch")
    dev = items[0][0].device
    descs, _ = _batch_descs(items, q)
    co = opts.to_c()
    co.single_site = 0
    n = len(items)
    nbytes = L.lib().plm_fit_batch_workspace_bytes(descs, n, q, ctypes.byref(co))
    if nbytes == 0:
        raise L.PlmError(L.PLM_E_INVALID, "invalid sizes or options")
    ws = workspace(nbytes, dev)
    res = (L.TuneResult * 16)()
    nout = ctypes.c_int32(0)
    ctx = context(dev)
    _check(L.lib().plm_tune(ctx, descs, n, q, ctypes.byref(co), int(bool(fp32_only)), _ptr(ws), ws.numel(),
                            res, 16, ctypes.byref(nout)), ctx)
    del ws
    return [dict(path=res[k].path, tile_seqs=res[k].tile_seqs, eval_ms=res[k].eval_ms)
            for k in range(nout.value)]


def last_fit_timing(device=None) -> dict:
    """Kernel times (ms) of the last fit run with timing=True on this device/stream."""
    ctx = context(device)
    t = L.FitTiming()
    _check(L.lib().plm_fit_last_timing(ctx, ctypes.byref(t)), ctx)
    return dict(forward_ms=t.forward_ms, backward_ms=t.backward_ms, lbfgs_ms=t.lbfgs_ms,
                total_ms=t.total_ms, iterations=int(t.iterations), site_evals=int(t.site_evals),
                quant_ms=t.quant_ms, refine_forward_ms=t.refine_forward_ms,
                refine_backward_ms=t.refine_backward_ms, refine_lbfgs_ms=t.refine_lbfgs_ms,
                refine_iterations=int(t.refine_iterations), refine_site_evals=int(t.refine_site_evals))


def score(J: torch.Tensor, combine: str = "avg", norm: str = "frob", p: float = 2.0,
          exclude_gap: bool = False, correction: str = "apc", freq: torch.Tensor | None = None):
    """(raw, corrected) float64 [N, N] pair scores (sec. 3.4 steps 4-6).

    The defaults give the paper's score: Frobenius norm of the averaged
    Ising-gauge couplings (FN) and its average-product correction (CFN).  The
    options select the variants of sec. 7: combine "avg" | "min" | "max",
    norm "frob" | "lp" (exponent p) | "burkoff" (needs freq, see
    frequencies()), exclude_gap, correction "apc" | "none" | "asc"."""
    dev = J.device
    _dev_tensor(J, torch.float32, dev, "J")
    N, _, q, _ = J.shape
    raw = torch.empty(N, N, dtype=torch.float64, device=dev)
    cor = torch.empty(N, N, dtype=torch.float64, device=dev)
    ctx = context(dev)
    default = (combine, norm, exclude_gap, correction) == ("avg", "frob", False, "apc")
    if default:
        _check(L.lib().plm_score(ctx, _ptr(J), N, q, _ptr(raw), _ptr(cor)), ctx)
        return raw, cor
    o = L.ScoreOpts()
    L.lib().plm_score_opts_default(ctypes.byref(o))
    o.combine = L.COMBINE[combine]
    o.norm = L.NORM[norm]
    o.p = float(p)
    o.exclude_gap = int(bool(exclude_gap))
    o.correction = L.CORRECTION[correction]
    if freq is not None:
        _dev_tensor(freq, torch.float64, dev, "freq")
        if tuple(freq.shape) != (N, q):
            raise ValueError("freq must be [N, q]")
    _check(L.lib().plm_score_ex(ctx, _ptr(J), N, q, ctypes.byref(o), _ptr(freq), _ptr(raw), _ptr(cor)), ctx)
    return raw, cor


def frequencies(msa, w, beff, q: int = 21) -> torch.Tensor:
    """Reweighted single-site frequencies float64 [N, q] on msa's device."""
    dev = msa.device
    _dev_tensor(msa, torch.uint8, dev, "msa")
    _dev_tensor(w, torch.float64, dev, "w")
    _dev_tensor(beff, torch.float64, dev, "beff")
    B, N = msa.shape
    f = torch.empty(N, q, dtype=torch.float64, device=dev)
    ctx = context(dev)
    _check(L.lib().plm_frequencies(ctx, _ptr(msa), B, N, q, _ptr(w), _ptr(beff), _ptr(f)), ctx)
    return f


def contact_tpr(scores: torch.Tensor, contacts: torch.Tensor, min_sep: int = 5, kmax: int | None = None):
    """True-positive rates (numpy float64) of the strongest pairs with j - i >= min_sep."""
    import numpy as np
    dev = scores.device
    _dev_tensor(scores, torch.float64, dev, "scores")
    N = scores.shape[0]
    c = contacts.to(device=dev, dtype=torch.uint8).contiguous()
    kmax = kmax or N * N
    out = np.zeros(kmax, dtype=np.float64)
    n = ctypes.c_int32(0)
    ctx = context(dev)
    _check(L.lib().plm_contact_tpr(ctx, _ptr(scores), N, _ptr(c), int(min_sep), int(kmax),
                                   out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(n)), ctx)
    return out[:n.value]


def parse_alignment(text, fmt: str = "auto"):
    """FASTA or Stockholm text (str or bytes) to a uint8 [B, N] numpy array of
    codes (A C D E F G H I K L M N P Q R S T V W Y = 0..19, gap = 20), inserts
    removed (sec. 4).  Host-side; move the result to the device with torch."""
    import numpy as np
    data = text.encode() if isinstance(text, str) else bytes(text)
    B, N = ctypes.c_int32(0), ctypes.c_int32(0)
    err = ctypes.create_string_buffer(512)
    rc = L.lib().plm_parse_alignment(data, len(data), L.FORMAT[fmt], None, 0, ctypes.byref(B), ctypes.byref(N),
                                     err, 512)
    if rc != 0:
        raise L.PlmError(rc, err.value.decode())
    out = np.zeros((B.value, N.value), dtype=np.uint8)
    rc = L.lib().plm_parse_alignment(data, len(data), L.FORMAT[fmt], out.ctypes.data_as(ctypes.c_void_p),
                                     out.size, ctypes.byref(B), ctypes.byref(N), err, 512)
    if rc != 0:
        raise L.PlmError(rc, err.value.decode())
    return out


def read_alignment(path: str, fmt: str = "auto"):
    """parse_alignment() of a file."""
    with open(path, "rb") as fh:
        return parse_alignment(fh.read(), fmt)
