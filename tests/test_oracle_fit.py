"""Pins for the oracle's per-site minimisation (sec. 3.4 step 3).  CPU only.

g_r^reg is strongly convex (log-sum-exp of affine maps plus an l2 term with
modulus mu = 2 min(lambda_h, lambda'_J)), so the minimiser is unique and any
correct optimiser must reach it; the pins are the optimum gauge identities of
sec. 3.2 (eq. asymmetricgauge), scikit-learn's multinomial logistic regression
(the paper calls each site problem one, sec. 3), scipy's L-BFGS-B, and the
distance certificate ||theta - theta*|| <= ||grad|| / mu."""
import math

import numpy as np
import pytest

import oracle
from oracle import brute


def _data(seed, B, N, q):
    rng = np.random.default_rng(seed)
    h, Jsym = brute.random_model(N, q, rng, 0.7, 0.6)
    # Gibbs-free: draw each row from the model by enumeration when small,
    # otherwise independent columns with a planted dependency
    if q ** N <= 5000:
        msa = brute.sample(h, Jsym, B, rng)
    else:
        msa = rng.integers(0, q, size=(B, N), dtype=np.uint8)
        msa[:, 1] = (msa[:, 0] + (rng.random(B) < 0.2)) % q
    w = rng.uniform(0.25, 1.0, size=B)
    return msa, w, float(w.sum())


def test_fit_converges_and_satisfies_optimum_gauge():
    N, q = 5, 4
    msa, w, beff = _data(1, 400, N, q)
    lh, lJ = 0.01, 0.01
    lJp = 0.5 * lJ
    h, J, stats = oracle.fit(msa, w, beff, lh, lJ, q=q, tol=1e-10)
    for t in range(N):
        assert stats[t]["status"] == 0 and stats[t]["gnorm"] <= 1e-10
        hr, Jr = h[t], J[t]
        assert abs(hr.sum()) < 1e-8
        for i in range(N):
            if i == t:
                assert np.all(Jr[i] == 0.0)
                continue
            # J[r][i][k][s] = J_ri(s,k): summed over s (state of r) is zero for each k
            np.testing.assert_allclose(Jr[i].sum(axis=1), 0.0, atol=1e-7)
            # lambda'_J * sum_k J_ri(s,k) = lambda_h h_r(s)
            np.testing.assert_allclose(lJp * Jr[i].sum(axis=0), lh * hr, atol=1e-9)


def test_fit_matches_sklearn_logistic_regression():
    sklearn = pytest.importorskip("sklearn.linear_model")
    N, q, B = 6, 4, 300
    msa, w, beff = _data(2, B, N, q)
    lh, lJ = 0.02, 0.01
    lJp = 0.5 * lJ
    c = math.sqrt(lJp / lh)
    h, J, stats = oracle.fit(msa, w, beff, lh, lJ, q=q, tol=1e-11)
    for r in (0, 2, 5):
        assert len(np.unique(msa[:, r])) == q
        others = [i for i in range(N) if i != r]
        X = np.zeros((B, 1 + len(others) * q))
        X[:, 0] = c
        for t, i in enumerate(others):
            X[np.arange(B), 1 + t * q + msa[:, i]] = 1.0
        # sklearn minimises C * sum_b w_b CE_b + 0.5 ||beta||^2 ; times 2 lambda'_J
        # this is the f/B_eff objective when C = 1 / (2 lambda'_J B_eff) and the
        # constant column carries h_r / c with c^2 = lambda'_J / lambda_h
        kw = dict(C=1.0 / (2.0 * lJp * beff), fit_intercept=False, tol=1e-12, max_iter=20000)
        try:
            clf = sklearn.LogisticRegression(solver="lbfgs", **kw)
        except TypeError:  # pragma: no cover
            clf = sklearn.LogisticRegression(solver="lbfgs", multi_class="multinomial", **kw)
        clf.fit(X, msa[:, r], sample_weight=w)
        coef = clf.coef_  # [q, features], classes 0..q-1 in order
        assert list(clf.classes_) == list(range(q))
        np.testing.assert_allclose(coef[:, 0] * c, h[r], atol=2e-6)
        for t, i in enumerate(others):
            # coef[s, (i,k)] = J_ri(s,k) = J[r][i][k][s]
            np.testing.assert_allclose(coef[:, 1 + t * q:1 + (t + 1) * q].T, J[r][i], atol=2e-6)


def test_fit_matches_scipy_lbfgsb():
    scipy_opt = pytest.importorskip("scipy.optimize")
    N, q = 4, 3
    msa, w, beff = _data(3, 200, N, q)
    lh, lJ = 0.01, 0.01
    h, J, stats = oracle.fit(msa, w, beff, lh, lJ, q=q, tol=1e-11)
    r = 1

    def fun(x):
        f, gh, gJ = oracle.site_objgrad(msa, r, w, beff, x[:q], x[q:].reshape(N, q, q), lh, lJ)
        return f / beff, np.concatenate([gh, gJ.ravel()]) / beff

    res = scipy_opt.minimize(fun, np.zeros(q + N * q * q), jac=True, method="L-BFGS-B",
                             options=dict(gtol=1e-12, ftol=1e-15, maxiter=20000))
    np.testing.assert_allclose(res.x[:q], h[r], atol=1e-6)
    np.testing.assert_allclose(res.x[q:].reshape(N, q, q), J[r], atol=1e-6)


def test_certificate_bounds_distance_to_optimum():
    N, q = 5, 3
    msa, w, beff = _data(4, 300, N, q)
    lh, lJ = 0.01, 0.01
    mu = 2 * min(lh, 0.5 * lJ)
    h_tight, J_tight, _ = oracle.fit(msa, w, beff, lh, lJ, q=q, tol=1e-12)
    h_loose, J_loose, st = oracle.fit(msa, w, beff, lh, lJ, q=q, tol=1e-3)
    for t in range(N):
        d = np.sqrt(np.sum((h_loose[t] - h_tight[t]) ** 2) + np.sum((J_loose[t] - J_tight[t]) ** 2))
        assert d <= st[t]["gnorm"] / mu + 1e-9


def test_consistency_recovers_true_couplings():
    # sec. 3: pseudolikelihood is a consistent estimator.  With many exact
    # samples and a tiny regulariser, the Ising-gauge couplings of each site
    # estimate approach those of the generating model.
    N, q, B = 3, 3, 40000
    rng = np.random.default_rng(12)
    h, Jsym = brute.random_model(N, q, rng, 0.5, 0.8)
    msa = brute.sample(h, Jsym, B, rng)
    w = np.ones(B)
    h_fit, J_fit, st = oracle.fit(msa, w, float(B), 1e-5, 1e-5, q=q, tol=1e-8)
    true = brute.ising_gauge_couplings(Jsym)
    for r in range(N):
        for i in range(N):
            if i == r:
                continue
            # site-r estimate as a (state of r, state of i) matrix
            A = J_fit[r][i].T
            A = A - A.mean(axis=0, keepdims=True) - A.mean(axis=1, keepdims=True) + A.mean()
            ref = true[r, i] if r < i else true[i, r].T
            assert np.max(np.abs(A - ref)) < 0.06
