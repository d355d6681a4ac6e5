"""FP64 oracle of the mean-field starting guess (sec. 2: couplings from the
inverse of the connected correlation matrix c_ij(k,l) = f_ij(k,l) -
f_i(k) f_j(l), made invertible by pseudocounts; sec. 7: used as a starting
point of the pseudolikelihood minimisation).  Test infrastructure only.

Readings (the paper names the method and its ingredients, not the formulas):
  * reweighted counts F_i(k) = sum_b w_b [sigma_i^b = k] and F_ij(k,l) =
    sum_b w_b [sigma_i^b = k][sigma_j^b = l], normalised by B_eff, are mixed
    with a uniform pseudocount of weight lam:
      f_i(k)    = (1 - lam) F_i(k) / B_eff + lam / q
      f_ij(k,l) = (1 - lam) F_ij(k,l) / B_eff + lam / q^2      (i != j)
      f_ii(k,l) = f_i(k) [k = l]
  * the last state (q - 1, the gap) is the reference: C is indexed by
    (i, k), k < q - 1, and the couplings and fields of the reference state
    are zero;
  * J_ij(k,l) = -(C^-1)_{(i,k),(j,l)} for i != j, self blocks zero;
  * fields from the mean-field equations with this gauge:
      h_i(k) = ln(f_i(k) / f_i(q-1)) - sum_{j != i} sum_{l < q-1} J_ij(k,l) f_j(l).
Storage: the asymmetric layout J[r][i][k][s] = J_ri(s, k) (s the state of r);
the mean-field model is consistent (J[i][r] is J[r][i] transposed).
Plain numpy, explicit per-pair loops for the frequencies.
"""
from __future__ import annotations

import numpy as np


def frequencies(msa, w, beff, q, lam):
    """(f_i [N, q], f_ij [N, N, q, q]) with pseudocounts; f_ii diagonal."""
    msa = np.asarray(msa)
    w = np.asarray(w, dtype=np.float64)
    B, N = msa.shape
    fi = np.zeros((N, q))
    for i in range(N):
        fi[i] = np.bincount(msa[:, i], weights=w, minlength=q)[:q]
    fi = (1.0 - lam) * fi / beff + lam / q
    fij = np.zeros((N, N, q, q))
    for i in range(N):
        for j in range(N):
            if i == j:
                fij[i, i] = np.diag(fi[i])
                continue
            cnt = np.bincount(msa[:, i].astype(np.int64) * q + msa[:, j], weights=w, minlength=q * q)[:q * q]
            fij[i, j] = (1.0 - lam) * cnt.reshape(q, q) / beff + lam / (q * q)
    return fi, fij


def correlation(fi, fij):
    """C [N(q-1), N(q-1)]: c_ij(k,l) = f_ij(k,l) - f_i(k) f_j(l), k, l < q - 1."""
    N, q = fi.shape
    r = q - 1
    C = np.zeros((N * r, N * r))
    for i in range(N):
        for j in range(N):
            C[i * r:(i + 1) * r, j * r:(j + 1) * r] = fij[i, j, :r, :r] - np.outer(fi[i, :r], fi[j, :r])
    return C


def inverse_correlation(msa, w, beff, q=21, lam=0.5):
    fi, fij = frequencies(msa, w, beff, q, lam)
    return fi, np.linalg.inv(correlation(fi, fij))


def couplings(msa, w, beff, q=21, lam=0.5):
    """(h [N, q], J [N, N, q, q]) of the mean-field model, asymmetric layout."""
    fi, Cinv = inverse_correlation(msa, w, beff, q, lam)
    N = fi.shape[0]
    r = q - 1
    J = np.zeros((N, N, q, q))
    for a in range(N):
        for i in range(N):
            if a == i:
                continue
            # J_ai(s, k) = -(C^-1)_{(a,s),(i,k)}; stored at J[a][i][k][s]
            J[a, i, :r, :r] = -Cinv[a * r:(a + 1) * r, i * r:(i + 1) * r].T
    h = np.zeros((N, q))
    for a in range(N):
        for s in range(r):
            t = np.log(fi[a, s] / fi[a, r])
            for i in range(N):
                if i != a:
                    t -= np.dot(J[a, i, :r, s], fi[i, :r])
            h[a, s] = t
    return h, J
