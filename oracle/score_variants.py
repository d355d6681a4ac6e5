"""FP64 oracle of the coupling-score variants the paper tried besides its
CFN score (sec. 7: min/max combinations of the two estimates, an l_p norm,
the Burkoff divergence of eqs. burkoffscore1/burkoffscore2, the gap state
left out of the norm, and the average-sum correction of eq. corr_normsum),
and of the true-positive rate of the strongest predicted contacts (sec. 6).

Test infrastructure only: tests and the benchmark's CPU leg use it, the
product path never does.  Plain numpy, one pair at a time.

Conventions (the paper's, eqs. gauge_change2 / average2 / frob_normtrans2):
J[r][i][k][s] holds J^{(r)}_{ri}(s, k); the two estimates of pair (i, j) as
q x q matrices indexed (state of i, state of j) are A = J[i][j]^T and
B = J[j][i]; each is moved to the Ising gauge (row and column means over all
q states subtracted, grand mean added) before they are combined.  States are
0..q-1 with the gap last (q-1).  Readings (not fixed by the paper): the l_p
norm sums |J|^p; the Burkoff score uses the combined Ising-gauge couplings
and the reweighted single-site frequencies; with the gap excluded the sums
run over states 0..q-2 of the Ising-gauge matrix computed with all q states.
"""
from __future__ import annotations

import numpy as np

COMBINE = ("avg", "min", "max")
NORMS = ("frob", "lp", "burkoff")
CORRECTIONS = ("apc", "none", "asc")


def ising_gauge(M):
    """M - row means - column means + grand mean (eq. gauge_change2)."""
    M = np.asarray(M, dtype=np.float64)
    return M - M.mean(axis=1, keepdims=True) - M.mean(axis=0, keepdims=True) + M.mean()


def pair_estimates(J, i, j):
    """(A, B): the site-i and site-j estimates of pair (i, j), (state i, state j)."""
    A = np.asarray(J[i, j], dtype=np.float64).T
    B = np.asarray(J[j, i], dtype=np.float64)
    return A, B


def combine(A, B, mode):
    Ag, Bg = ising_gauge(A), ising_gauge(B)
    if mode == "avg":
        return 0.5 * (Ag + Bg)
    if mode == "min":
        return np.minimum(Ag, Bg)
    if mode == "max":
        return np.maximum(Ag, Bg)
    raise ValueError(mode)


def frequencies(msa, w, beff, q):
    """Reweighted single-site frequencies f_i(k) = sum_b w_b [sigma_i^b = k] / B_eff."""
    msa = np.asarray(msa)
    B, N = msa.shape
    f = np.zeros((N, q))
    for i in range(N):
        f[i] = np.bincount(msa[:, i], weights=np.asarray(w, dtype=np.float64), minlength=q)[:q]
    return f / beff


def pair_norm(M, norm, p=2.0, exclude_gap=False, fi=None, fj=None):
    q = M.shape[0]
    sl = slice(0, q - 1) if exclude_gap else slice(0, q)
    Ms = M[sl, sl]
    if norm == "frob":
        return float(np.sqrt(np.sum(Ms * Ms)))
    if norm == "lp":
        return float(np.sum(np.abs(Ms) ** p) ** (1.0 / p))
    if norm == "burkoff":
        # P(k,l) proportional to f_i(k) f_j(l) exp(J(k,l)); D = sum P ln(P / (f_i f_j))
        ff = np.outer(fi[sl], fj[sl])
        wts = ff * np.exp(Ms)
        Z = wts.sum()
        if Z <= 0.0:
            return 0.0
        P = wts / Z
        nz = P > 0
        return float(np.sum(P[nz] * (Ms[nz] - np.log(Z))))
    raise ValueError(norm)


def raw_scores(J, combine_mode="avg", norm="frob", p=2.0, exclude_gap=False, freq=None):
    """N x N symmetric raw pair scores, zero diagonal."""
    J = np.asarray(J)
    N = J.shape[0]
    S = np.zeros((N, N))
    for i in range(N):
        for j in range(i + 1, N):
            A, B = pair_estimates(J, i, j)
            M = combine(A, B, combine_mode)
            v = pair_norm(M, norm, p, exclude_gap,
                          None if freq is None else freq[i], None if freq is None else freq[j])
            S[i, j] = S[j, i] = v
    return S


def correct(S, mode):
    """Correction of an N x N raw score matrix with zero diagonal; means over
    all N positions (diagonal zeros included); the corrected diagonal is 0."""
    S = np.asarray(S, dtype=np.float64)
    N = S.shape[0]
    r = S.mean(axis=1)
    c = S.mean(axis=0)
    a = S.mean()
    if mode == "none":
        out = S.copy()
    elif mode == "apc":
        out = S - np.outer(r, c) / a if a != 0.0 else np.zeros_like(S)
    elif mode == "asc":
        out = S - r[:, None] - c[None, :] + a
    else:
        raise ValueError(mode)
    out[np.arange(N), np.arange(N)] = 0.0
    return out


def tpr_curve(S, contacts, min_sep=5, kmax=None):
    """True-positive rate of the k strongest pairs with |i - j| >= min_sep,
    k = 1..kmax: ranked by decreasing score, ties by (i, j)."""
    S = np.asarray(S)
    N = S.shape[0]
    cand = [(i, j) for i in range(N) for j in range(i + min_sep, N)]
    cand.sort(key=lambda ij: (-S[ij[0], ij[1]], ij[0], ij[1]))
    kmax = len(cand) if kmax is None else min(kmax, len(cand))
    hits = 0
    out = np.zeros(kmax)
    for k in range(kmax):
        i, j = cand[k]
        hits += 1 if contacts[i, j] else 0
        out[k] = hits / (k + 1)
    return out
