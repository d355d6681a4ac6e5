"""Pins of the mean-field oracle: the weak-coupling limit of an exactly
enumerated Potts model (mean-field couplings and fields are exact to first
order in J, in the gauge with the last state as reference), closed forms for
product alignments with and without pseudocounts, the mean-field equations
at the returned fields, and consistency of the two stored estimates."""
import itertools

import numpy as np

from oracle import meanfield as mf


def _exact_marginal_alignment(h, J):
    """All q^N configurations of a Potts model, weighted by their exact
    probabilities (so the weighted frequencies are the exact marginals).
    h [N, q]; J[i][j][k][l] = J_ij(k, l) for i < j (state k at i, l at j)."""
    N, q = h.shape
    confs = np.array(list(itertools.product(range(q), repeat=N)), dtype=np.uint8)
    E = np.zeros(len(confs))
    for c, x in enumerate(confs):
        e = sum(h[i, x[i]] for i in range(N))
        for i in range(N):
            for j in range(i + 1, N):
                e += J[i, j, x[i], x[j]]
        E[c] = e
    p = np.exp(E - E.max())
    p /= p.sum()
    return confs, p


def _reference_gauge(h, J):
    """Fields and couplings with the last state as reference:
    J'_ij(k,l) = J(k,l) - J(k,q) - J(q,l) + J(q,q), h'_i(k) = h_i(k) - h_i(q)
    + sum_{j != i} [J_ij(k, q) - J_ij(q, q)], in the asymmetric layout."""
    N, q = h.shape
    r = q - 1

    def Jij(i, j):  # (state of i, state of j)
        return J[i, j] if i < j else J[j, i].T

    Jl = np.zeros((N, N, q, q))
    hl = np.zeros((N, q))
    for a in range(N):
        hl[a] = h[a] - h[a, r]
        for i in range(N):
            if i == a:
                continue
            M = Jij(a, i)
            Mp = M - M[:, [r]] - M[[r], :] + M[r, r]
            Jl[a, i] = Mp.T  # J[a][i][k][s] = J_ai(s, k)
            hl[a] += M[:, r] - M[r, r]
    hl -= hl[:, [r]]
    return hl, Jl


def test_weak_coupling_limit_is_exact_to_first_order():
    N, q = 3, 3
    rng = np.random.default_rng(0)
    h = 0.5 * rng.standard_normal((N, q))
    G = rng.standard_normal((N, N, q, q))  # not symmetric in (k, l): pins the transpose
    errs = []
    for eps in (0.02, 0.04):
        J = eps * G
        confs, p = _exact_marginal_alignment(h, J)
        hm, Jm = mf.couplings(confs, p, 1.0, q=q, lam=0.0)
        hl, Jl = _reference_gauge(h, J)
        eJ = np.max(np.abs(Jm - Jl))
        eh = np.max(np.abs(hm - hl))
        errs.append((eJ, eh))
        assert eJ <= 4 * eps ** 2 and eh <= 4 * eps ** 2, (eps, eJ, eh)
        # first order really is captured: the coupling itself is much larger than the error
        assert np.max(np.abs(Jl)) >= 10 * eJ
    # the error is second order: doubling eps multiplies it by about 4
    for k in range(2):
        ratio = errs[1][k] / errs[0][k]
        assert 3.0 <= ratio <= 5.0, (k, ratio)


def _product_alignment(cols):
    """Every combination of the given column multisets: pair frequencies
    factorise exactly, f_ij = f_i f_j (uniform weights)."""
    rows = np.array(list(itertools.product(*cols)), dtype=np.uint8)
    return rows, np.ones(len(rows))


def test_product_alignment_without_pseudocount_is_independent_sites():
    cols = [[0, 0, 1, 2, 3], [3, 1, 1, 2, 0, 0], [2, 0, 1, 3]]
    q = 4
    msa, w = _product_alignment(cols)
    h, J = mf.couplings(msa, w, float(w.sum()), q=q, lam=0.0)
    assert np.max(np.abs(J)) <= 1e-11
    for i, c in enumerate(cols):
        f = np.bincount(c, minlength=q) / len(c)
        np.testing.assert_allclose(h[i], np.log(f / f[q - 1]), rtol=0, atol=1e-12)


def test_pseudocount_correlation_closed_form():
    # with f_ij^data = f_i^data f_j^data, the pseudocounts alone give
    # c_ij(k,l) = lam (1 - lam) (f_i(k) - 1/q) (f_j(l) - 1/q) for i != j
    cols = [[0, 0, 1, 2, 3], [3, 1, 1, 2, 0, 0], [2, 0, 1, 3]]
    q, lam = 4, 0.3
    msa, w = _product_alignment(cols)
    fi, fij = mf.frequencies(msa, w, float(w.sum()), q, lam)
    C = mf.correlation(fi, fij)
    fd = [np.bincount(c, minlength=q) / len(c) for c in cols]
    r = q - 1
    for i in range(3):
        for j in range(3):
            blk = C[i * r:(i + 1) * r, j * r:(j + 1) * r]
            if i == j:
                f = (1 - lam) * fd[i] + lam / q
                expect = np.diag(f[:r]) - np.outer(f[:r], f[:r])
            else:
                expect = lam * (1 - lam) * np.outer(fd[i][:r] - 1 / q, fd[j][:r] - 1 / q)
            np.testing.assert_allclose(blk, expect, rtol=0, atol=1e-15)


def test_full_pseudocount_gives_the_uniform_model():
    rng = np.random.default_rng(1)
    msa = rng.integers(0, 5, size=(40, 6), dtype=np.uint8)
    h, J = mf.couplings(msa, np.ones(40), 40.0, q=5, lam=1.0)
    assert np.max(np.abs(J)) <= 1e-12 and np.max(np.abs(h)) <= 1e-12


def test_fields_solve_the_mean_field_equations_and_estimates_are_consistent():
    rng = np.random.default_rng(2)
    N, q = 7, 5
    msa = rng.integers(0, q, size=(120, N), dtype=np.uint8)
    msa[:, 3] = (msa[:, 1] + rng.integers(0, 2, size=120)) % q  # a correlated pair
    w = rng.uniform(0.2, 1.0, size=120)
    lam = 0.5
    h, J = mf.couplings(msa, w, float(w.sum()), q=q, lam=lam)
    fi, _ = mf.frequencies(msa, w, float(w.sum()), q, lam)
    for a in range(N):
        # f_a(s) is proportional to exp(h_a(s) + sum_i sum_k J_ai(s, k) f_i(k))
        field = h[a].copy()
        for i in range(N):
            if i != a:
                field += J[a, i].T @ fi[i]
        m = np.exp(field - field.max())
        np.testing.assert_allclose(m / m.sum(), fi[a], rtol=1e-12, atol=0)
        for i in range(N):
            np.testing.assert_allclose(J[i, a], J[a, i].T, rtol=1e-12, atol=1e-14)
    assert np.max(np.abs(J[1, 3])) > 10 * np.median(np.abs(J[0, 5]))  # the planted pair stands out
