"""Seeded synthetic alignments sampled from planted Potts models.

Stand-ins for the protein families the paper uses (PFAM alignments are not
available here): q = 21 symbols (20 amino acids + gap, gap = 20), N columns,
B rows, Gibbs-sampled from a Potts model with N(0,1) fields and a set of
planted pairs whose q x q coupling blocks are N(0, 0.5^2); all other couplings
are zero.  Shared by the tests and the benchmark; holds none of the inference
method's arithmetic.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libplm_synth.so")
_CACHE = os.path.join(os.path.dirname(_HERE), ".cache", "synth")
GAP = 20
Q = 21


def build(force: bool = True) -> str:
    """Compile the generator with the host C compiler (portable x86-64 code)."""
    if force or not os.path.exists(_SO):
        src = os.path.join(_HERE, "potts_gen.c")
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c99", "-ffp-contract=off",
                               "-o", tmp, src, "-lm", "-lpthread"])
        os.replace(tmp, _SO)
    return _SO


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        build(force=not os.path.exists(_SO))
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        L.synth_potts_model.restype = ctypes.c_int
        L.synth_potts_model.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_double, ctypes.c_double, P, P, P]
        L.synth_gibbs.restype = None
        L.synth_gibbs.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int, P, ctypes.c_int, P, P,
                                  ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, ctypes.c_int]
        L.synth_force_gaps.restype = None
        L.synth_force_gaps.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                       ctypes.c_uint8, P]
        L.synth_uniform.restype = None
        L.synth_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, P]
        _lib_handle = L
    return _lib_handle


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def uniform(seed: int, stream: int, n: int) -> np.ndarray:
    """n seeded uniform draws in [0, 1) (xoshiro256** stream (seed, stream))."""
    out = np.empty(n, dtype=np.float64)
    _lib().synth_uniform(seed, stream, n, _ptr(out))
    return out


@dataclass
class SynthMSA:
    name: str
    msa: np.ndarray            # uint8 [B, N]
    h: np.ndarray              # float64 [N, q] true fields
    pairs: np.ndarray          # int32 [P, 2] planted pairs (i < j)
    Jp: np.ndarray             # float64 [P, q, q] planted blocks (state of i, state of j)
    seed: int
    uniform_weights: bool = False
    theta: float = 0.8
    lambda_h: float = 0.01
    lambda_J: float = 0.01
    meta: dict = field(default_factory=dict)

    @property
    def B(self) -> int:
        return int(self.msa.shape[0])

    @property
    def N(self) -> int:
        return int(self.msa.shape[1])

    q: int = Q


def _threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except Exception:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def make_msa(name: str, N: int, B: int, npairs: int, seed: int, min_sep: int = 5,
             gap_p: float = 0.0, q: int = Q, nchains: int = 64, burnin: int = 1000,
             thin: int = 10, h_sd: float = 1.0, j_sd: float = 0.5, cache: bool = True,
             **kw) -> SynthMSA:
    key = f"{name}_N{N}_B{B}_P{npairs}_s{seed}_m{min_sep}_g{gap_p}_q{q}_c{nchains}_b{burnin}_t{thin}"
    path = os.path.join(_CACHE, key + ".npz")
    if cache and os.path.exists(path):
        z = np.load(path, allow_pickle=False)
        return SynthMSA(name, z["msa"], z["h"], z["pairs"], z["Jp"], seed, **kw)
    L = _lib()
    h = np.zeros((N, q), dtype=np.float64)
    pairs = np.zeros((max(npairs, 1), 2), dtype=np.int32)
    Jp = np.zeros((max(npairs, 1), q, q), dtype=np.float64)
    got = L.synth_potts_model(seed, N, q, npairs, min_sep, h_sd, j_sd, _ptr(h), _ptr(pairs), _ptr(Jp))
    pairs = np.ascontiguousarray(pairs[:got])
    Jp = np.ascontiguousarray(Jp[:got])
    msa = np.zeros((B, N), dtype=np.uint8)
    L.synth_gibbs(seed, N, q, _ptr(h), got, _ptr(pairs), _ptr(Jp), B, nchains, burnin, thin,
                  _ptr(msa), _threads())
    if gap_p > 0.0:
        L.synth_force_gaps(seed, B, N, gap_p, GAP, _ptr(msa))
    if cache:
        os.makedirs(_CACHE, exist_ok=True)
        tmp = path + ".tmp%d.npz" % os.getpid()
        np.savez(tmp, msa=msa, h=h, pairs=pairs, Jp=Jp)
        os.replace(tmp, path)
    return SynthMSA(name, msa, h, pairs, Jp, seed, **kw)


# The benchmark workloads: sizes and structure of the paper's families
# (N 50-500, B up to ~1e5, q = 21, gap-rich columns).
WORKLOADS = {
    # plain FP64 fit at the smallest size, uniform weights, planted pairs anywhere
    "potts_n40_b500": dict(N=40, B=500, npairs=80, seed=1, min_sep=1, uniform_weights=True),
    # all-sites batched fit with 10% forced gaps and 0.8-identity reweighting
    "potts_n120_b5000_gaps": dict(N=120, B=5000, npairs=240, seed=2, min_sep=5, gap_p=0.1),
    # autograd checks
    "potts_n150_b8000": dict(N=150, B=8000, npairs=300, seed=3, min_sep=5),
    # the large fit
    "potts_n500_b50000": dict(N=500, B=50000, npairs=2000, seed=5, min_sep=5),
}


def workload(name: str, **over) -> SynthMSA:
    cfg = dict(WORKLOADS[name])
    cfg.update(over)
    return make_msa(name, **cfg)


def ragged_set(count: int = 16, seed: int = 4, n_range=(60, 300), b_range=(2000, 30000),
               **over) -> list:
    """`count` alignments with N, B drawn uniformly from the given integer
    ranges (seeded), 2N planted pairs each, seeds 400 + k."""
    u = uniform(seed, 77, 2 * count)
    out = []
    for k in range(count):
        N = n_range[0] + int(u[2 * k] * (n_range[1] - n_range[0] + 1))
        B = b_range[0] + int(u[2 * k + 1] * (b_range[1] - b_range[0] + 1))
        N = min(N, n_range[1])
        B = min(B, b_range[1])
        cfg = dict(N=N, B=B, npairs=2 * N, seed=400 + k, min_sep=5)
        cfg.update(over)
        out.append(make_msa(f"ragged{k}", **cfg))
    return out


def sample_sites(seed: int, N: int, k: int) -> list:
    """k distinct site indices drawn uniformly from 0..N-1 (partial
    Fisher-Yates shuffle on the seeded stream (seed, 55)), sorted."""
    u = uniform(seed, 55, k)
    idx = list(range(N))
    for t in range(k):
        j = t + min(int(u[t] * (N - t)), N - t - 1)
        idx[t], idx[j] = idx[j], idx[t]
    return sorted(idx[:k])


def msa_digest(msa: np.ndarray) -> str:
    """SHA-256 of an alignment's bytes and shape (identifies stored fixtures)."""
    import hashlib
    a = np.ascontiguousarray(msa, dtype=np.uint8)
    h = hashlib.sha256()
    h.update(np.asarray(a.shape, dtype=np.int64).tobytes())
    h.update(a.tobytes())
    return h.hexdigest()
