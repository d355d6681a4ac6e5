"""Pins of the symmetric-PLM oracle: central differences of F, the gauge
the l2 penalty implies at the optimum (eq. symmetricgauge), and agreement
of F with the per-site objectives summed (with lambda'_J = lambda_J / 2
each pair's penalty is counted once, as in eq. l2reg)."""
import numpy as np

import oracle
from oracle import symmetric as sym
from tests.helpers import clustered_msa


def _problem(seed=0, B=300, N=6, q=4):
    rng = np.random.default_rng(seed)
    msa = rng.integers(0, q, size=(B, N), dtype=np.uint8)
    w = rng.uniform(0.3, 1.0, size=B)
    return msa, w, float(w.sum())


def test_gradient_matches_central_differences():
    msa, w, beff = _problem()
    N, q = 6, 4
    rng = np.random.default_rng(1)
    h = 0.3 * rng.standard_normal((N, q))
    J = sym.mirror(0.3 * rng.standard_normal((N, N, q, q)))
    F, gh, gJ = sym.objective(msa, w, beff, h, J)
    eps = 1e-6
    for _ in range(25):
        if rng.random() < 0.3:
            r, k = rng.integers(N), rng.integers(q)
            hp, hm = h.copy(), h.copy()
            hp[r, k] += eps
            hm[r, k] -= eps
            fd = (sym.objective(msa, w, beff, hp, J)[0] - sym.objective(msa, w, beff, hm, J)[0]) / (2 * eps)
            assert abs(fd - gh[r, k]) <= 1e-7, (fd, gh[r, k])
        else:
            i, j = sorted(rng.choice(N, 2, replace=False))
            k, s = rng.integers(q), rng.integers(q)
            Jp, Jm = J.copy(), J.copy()
            Jp[i, j, k, s] += eps
            Jm[i, j, k, s] -= eps
            fd = (sym.objective(msa, w, beff, h, Jp)[0] - sym.objective(msa, w, beff, h, Jm)[0]) / (2 * eps)
            assert abs(fd - gJ[i, j, k, s]) <= 1e-7, (fd, gJ[i, j, k, s])


def test_objective_is_the_sum_of_site_objectives_for_shared_couplings():
    msa, w, beff = _problem(seed=2)
    rng = np.random.default_rng(3)
    N, q = 6, 4
    h = 0.2 * rng.standard_normal((N, q))
    J = sym.mirror(0.2 * rng.standard_normal((N, N, q, q)))
    F, _, _ = sym.objective(msa, w, beff, h, J, 0.02, 0.03)
    f, _, _ = oracle.objgrad(msa, w, beff, h, J, 0.02, 0.03)  # per-site penalty lambda_J / 2
    assert abs(F - f.sum() / beff) <= 1e-12 * abs(F)


def test_fit_satisfies_the_symmetric_gauge():
    msa = clustered_msa(seed=5, B=400, N=7, n_anc=4, p_mut=0.3)
    msa = (msa % 5).astype(np.uint8)
    w = np.ones(msa.shape[0])
    lh, lJ = 0.01, 0.02
    h, J, gn = sym.fit(msa, w, float(msa.shape[0]), lh, lJ, q=5)
    assert gn <= 1e-7, gn  # distance to the optimum <= gn / (2 min(lambda_h, lambda_J)) = 2.5e-6
    N = msa.shape[1]
    # lambda_J sum_s J_ij(k, s) = lambda_h h_i(k) for every j != i (sum over the state of j),
    # and sum_k h_i(k) = 0; J[i][j][kj][si] holds J_ij(si, kj).  The residuals move by at most
    # (lambda_J sqrt(q) + lambda_h) times the distance to the optimum.
    tol = 2e-7
    for i in range(N):
        assert abs(h[i].sum()) <= tol
        for j in range(N):
            if j != i:
                row = lJ * J[i, j].sum(axis=0)  # sum over the state of j, indexed by the state of i
                assert np.max(np.abs(row - lh * h[i])) <= tol, (i, j, np.max(np.abs(row - lh * h[i])))
