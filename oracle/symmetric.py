"""FP64 oracle of symmetric pseudolikelihood maximization (eqs. npll_1 and
l2reg): one minimisation of F = sum_r g_r + lambda_h sum_i ||h_i||^2 +
lambda_J sum_{i<j} ||J_ij||^2 with each J_ij shared by g_i and g_j.  Test
infrastructure only.

Storage: the asymmetric layout J[r][i][k][s] = J_ri(s, k) (s the state of r),
filled consistently: J[j][i] is J[i][j] with its two state axes swapped.
The independent parameters are h and the blocks J[i][j], i < j.  The data
part of F and its gradient come from the pinned per-site oracle (all sites,
no regulariser); the gradient of a shared block is the sum of the site-i
and site-j gradients (the latter transposed).  The minimiser is unique
(strongly convex), computed with scipy's L-BFGS-B to a tight tolerance and
certified by the gradient norm at the returned point.
"""
from __future__ import annotations

import numpy as np

import oracle


def mirror(J):
    """J with J[j][i] set to the transpose of J[i][j] for i < j (self blocks zero)."""
    J = np.array(J, dtype=np.float64, copy=True)
    N = J.shape[0]
    for i in range(N):
        J[i, i] = 0.0
        for j in range(i + 1, N):
            J[j, i] = J[i, j].T
    return J


def objective(msa, w, beff, h, J, lambda_h=0.01, lambda_J=0.01):
    """F (normalised), dF/dh [N, q], dF/dJ on the blocks i < j (others zero)."""
    J = mirror(J)
    N = J.shape[0]
    f, gh_d, gJ_d = oracle.objgrad(msa, w, beff, h, J, 0.0, 0.0)
    iu = np.triu_indices(N, 1)
    F = f.sum() / beff + lambda_h * np.sum(h * h) + lambda_J * np.sum(J[iu] ** 2)
    gh = gh_d / beff + 2 * lambda_h * h
    gJ = np.zeros_like(J)
    for i in range(N):
        for j in range(i + 1, N):
            gJ[i, j] = (gJ_d[i, j] + gJ_d[j, i].T) / beff + 2 * lambda_J * J[i, j]
    return F, gh, gJ


def _pack(h, J):
    N = J.shape[0]
    iu = np.triu_indices(N, 1)
    return np.concatenate([h.ravel(), J[iu].ravel()])


def _unpack(x, N, q):
    h = x[:N * q].reshape(N, q)
    J = np.zeros((N, N, q, q))
    iu = np.triu_indices(N, 1)
    J[iu] = x[N * q:].reshape(len(iu[0]), q, q)
    return h, mirror(J)


def fit(msa, w, beff, lambda_h=0.01, lambda_J=0.01, q=21, gtol=1e-10, max_iter=20000):
    """(h, J, gnorm): the symmetric minimiser (J mirrored) and the Euclidean
    norm of the gradient of F there."""
    from scipy.optimize import minimize
    N = np.asarray(msa).shape[1]

    def fun(x):
        h, J = _unpack(x, N, q)
        F, gh, gJ = objective(msa, w, beff, h, J, lambda_h, lambda_J)
        return F, _pack(gh, gJ)

    x0 = np.zeros(N * q + N * (N - 1) // 2 * q * q)
    res = minimize(fun, x0, jac=True, method="L-BFGS-B",
                   options=dict(maxiter=max_iter, maxcor=20, gtol=gtol, ftol=1e-16))
    h, J = _unpack(res.x, N, q)
    _, gh, gJ = objective(msa, w, beff, h, J, lambda_h, lambda_J)
    gn = float(np.sqrt(np.sum(gh ** 2) + np.sum(gJ ** 2)))
    return h, J, gn
