"""Cache of the autotuner's choices: the fastest evaluation schedule (path and
forward tile size) per size bucket of a batch.

The timing itself runs in the library (plm_tune: every candidate schedule on
the caller's own alignments, HIP events on the device).  This module keys the
result by device, q, precision class and the (N, B) bucket of every alignment
-- ceil(log2 N), ceil(log2 B) -- and keeps it in a JSON file
($PLM_TUNE_CACHE, else ~/.cache/paper_1401_4832_amd/tune.json), so that later
fits of similar sizes reuse it without timing again."""
from __future__ import annotations

import dataclasses
import json
import math
import os

import torch

from . import api


def cache_path() -> str:
    return os.environ.get("PLM_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_1401_4832_amd", "tune.json"))


def bucket(N: int, B: int) -> tuple:
    return (int(math.ceil(math.log2(max(N, 2)))), int(math.ceil(math.log2(max(B, 2)))))


def _arch(dev) -> str:
    return getattr(torch.cuda.get_device_properties(dev), "gcnArchName", "gpu").split(":")[0]


# the fixed-point evaluation paths: residuals (and on path 6 couplings) rounded
# on a fixed grid, with exact integer sums
FIXED_POINT_PATHS = (5, 6)


def fixed_point_floor(item, q: int) -> float:
    """Expected size of the per-site gradient norm (B_eff-normalised) that the
    rounding of the residuals to 2^-23 leaves on the fixed-point paths: each of
    the N q^2 coupling entries sums B rounding errors of standard deviation
    2^-23 / sqrt(3)."""
    if len(item) < 3:
        return 0.0
    msa, _, beff = item
    B, N = int(msa.shape[0]), int(msa.shape[1])
    be = float(beff.item()) if hasattr(beff, "item") else float(beff)
    return 2.0 ** -23 * math.sqrt(N * q * q * B / 3.0) / max(be, 1e-300)


def symmetric_floor(item, q: int) -> float:
    """The same estimate for the symmetric fit, whose gradient norm runs over
    all N q + N (N - 1) / 2 q^2 parameters (each coupling block's gradient is
    the sum of two sites' sums)."""
    if len(item) < 3:
        return 0.0
    msa, _, beff = item
    B, N = int(msa.shape[0]), int(msa.shape[1])
    be = float(beff.item()) if hasattr(beff, "item") else float(beff)
    P = N * q + N * (N - 1) // 2 * q * q
    return 2.0 ** -23 * math.sqrt(P * B / 3.0) / max(be, 1e-300)


def key(items, q: int, fp32_only: bool, fixed_point: bool = True, symmetric: bool = False) -> str:
    arch = _arch(items[0][0].device)
    bs = sorted(bucket(int(it[0].shape[1]), int(it[0].shape[0])) for it in items)
    cls = ("fp32" if fp32_only else "any") + ("-sym" if symmetric else "") + ("" if fixed_point else "-nofixed")
    return f"{arch}|q{q}|{cls}|" + ",".join(f"{n}x{b}" for n, b in bs)


def load(path: str | None = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as fh:
            d = json.load(fh)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def store(d: dict, path: str | None = None) -> None:
    path = path or cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as fh:
        json.dump(d, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def choose(items, opts=None, q: int = 21, fp32_only: bool = True, path: str | None = None,
           retune: bool = False, fixed_point: bool = True, symmetric: bool = False) -> dict:
    """The cached schedule for this batch's bucket, timing the candidates on
    the batch itself on a miss (or when retune is set).  The fixed-point paths
    are candidates only where the expected gradient norm their residual
    rounding leaves is below half the tolerance (fixed_point=False leaves
    them out).  For the symmetric fit (symmetric=True) that norm runs over all
    parameters, and only the path with FP32 energies (5) is a candidate: its
    fit is refined on an FP32-class path; the rounded couplings of path 6
    move the symmetric gradient by more than such tolerances."""
    opts = opts or api.FitOptions()
    floor = symmetric_floor if symmetric else fixed_point_floor
    fixed_point = fixed_point and all(floor(it, q) * 2.0 < opts.tol for it in items)
    k = key(items, q, fp32_only, fixed_point, symmetric)
    d = load(path)
    if not retune and k in d:
        return d[k]
    res = api.tune(items, opts, q, fp32_only)
    if not fixed_point:
        res = [r for r in res if r["path"] not in FIXED_POINT_PATHS]
    elif symmetric:
        res = [r for r in res if r["path"] != 6]
    entry = dict(path=res[0]["path"], tile_seqs=res[0]["tile_seqs"], eval_ms=res[0]["eval_ms"],
                 candidates=res)
    d = load(path)  # re-read: another process may have written meanwhile
    d[k] = entry
    store(d, path)
    return entry


def tuned_options(items, opts, q: int = 21, fixed_point: bool = True, symmetric: bool = False):
    """opts with path and tile_seqs taken from the tuner (autotune cleared)."""
    ch = choose(items, opts, q, fixed_point=fixed_point, symmetric=symmetric)
    return dataclasses.replace(opts, path=int(ch["path"]), tile_seqs=int(ch["tile_seqs"]), autotune=False)
