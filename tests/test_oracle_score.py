"""Pins for the oracle's scoring (sec. 3.4 steps 4-6: eqs. gauge_change2,
average2, frob_normtrans2, corr_norm2).  CPU only."""
import numpy as np
import pytest

import oracle
from oracle import brute


def _sym_to_site_layout(Jsym):
    """Per-site layout J[r][i][k][s] = J_ri(s,k) from a symmetric model in which
    both sites see the same coupling (J_ri(s,k) = Jsym[r,i,s,k] for r < i)."""
    N, _, q, _ = Jsym.shape
    J = np.zeros((N, N, q, q))
    for r in range(N):
        for i in range(N):
            if i == r:
                continue
            A = Jsym[r, i] if r < i else Jsym[i, r].T  # (state of r, state of i)
            J[r, i] = A.T
    return J


def test_consistent_estimates_give_ising_gauge_norm():
    # when both estimates of every pair are the same coupling (the symmetric
    # case of sec. 2), the average is that coupling, and FN is the Frobenius
    # norm of its double-centred (Ising gauge) form.  A missing transpose of
    # the partner estimate breaks this for non-symmetric blocks.
    rng = np.random.default_rng(0)
    N, q = 5, 4
    _, Jsym = brute.random_model(N, q, rng, 1.0, 1.0)
    fn, cfn = oracle.score(_sym_to_site_layout(Jsym))
    ising = brute.ising_gauge_couplings(Jsym)
    for i in range(N):
        assert fn[i, i] == 0.0 and cfn[i, i] == 0.0
        for j in range(i + 1, N):
            assert fn[i, j] == pytest.approx(np.sqrt(np.sum(ising[i, j] ** 2)), rel=1e-12)
            assert fn[j, i] == fn[i, j]


def test_fn_is_gauge_invariant_and_minimal():
    # adding u(s) + v(k) to any block leaves FN unchanged (gauge freedom of
    # sec. 3.2), and the Ising gauge has the smallest norm (sec. 3.3)
    rng = np.random.default_rng(1)
    N, q = 6, 5
    J = rng.standard_normal((N, N, q, q))
    for r in range(N):
        J[r, r] = 0
    fn0, cfn0 = oracle.score(J)
    J2 = J.copy()
    for r in range(N):
        for i in range(N):
            if i != r:
                J2[r, i] += rng.standard_normal(q)[:, None] + rng.standard_normal(q)[None, :]
    fn1, cfn1 = oracle.score(J2)
    np.testing.assert_allclose(fn1, fn0, rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(cfn1, cfn0, rtol=1e-10, atol=1e-11)
    for i in range(N):
        for j in range(i + 1, N):
            raw = 0.5 * (J[i, j].T + J[j, i])  # both as (state of i, state of j)
            assert fn0[i, j] <= np.sqrt(np.sum(raw ** 2)) + 1e-12


def test_apc_closed_form_for_rank_one_norms():
    # blocks a_i a_j U with U double-centred and unit norm give FN_ij = a_i a_j
    # (i != j) and FN_ii = 0; with position averages over all N entries
    # (denominators N and N^2) the corrected score has a closed form
    rng = np.random.default_rng(2)
    N, q = 7, 3
    U = rng.standard_normal((q, q))
    U = U - U.mean(0, keepdims=True) - U.mean(1, keepdims=True) + U.mean()
    U /= np.sqrt(np.sum(U ** 2))
    a = rng.uniform(0.5, 2.0, size=N)
    Jsym = np.zeros((N, N, q, q))
    for i in range(N):
        for j in range(i + 1, N):
            Jsym[i, j] = a[i] * a[j] * U
    fn, cfn = oracle.score(_sym_to_site_layout(Jsym))
    A, A2 = a.sum(), np.sum(a ** 2)
    for i in range(N):
        for j in range(N):
            if i == j:
                continue
            assert fn[i, j] == pytest.approx(a[i] * a[j], rel=1e-12)
            rowi = a[i] * (A - a[i]) / N
            rowj = a[j] * (A - a[j]) / N
            allm = (A * A - A2) / (N * N)
            assert cfn[i, j] == pytest.approx(a[i] * a[j] - rowi * rowj / allm, rel=1e-11, abs=1e-13)


def test_float32_input_path_equals_double_path():
    rng = np.random.default_rng(3)
    J = rng.standard_normal((5, 5, 4, 4)).astype(np.float32)
    a = oracle.score(J)
    b = oracle.score(J.astype(np.float64))
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_planted_pairs_rank_first():
    # whole-method sanity on a small planted instance: fit every site, score,
    # and the strongest pairs are the planted ones (sec. 5 uses top-ranked pairs)
    import synth
    s = synth.make_msa("oracle_recovery", N=14, B=2500, npairs=4, seed=21, min_sep=3,
                       j_sd=1.0, cache=False)
    m, w, beff = oracle.reweight(s.msa, theta=0.8)
    h, J, st = oracle.fit(s.msa, w, beff, 0.01, 0.01, tol=1e-6)
    fn, cfn = oracle.score(J)
    iu = np.triu_indices(14, 1)
    order = np.argsort(-cfn[iu])
    top = {(int(iu[0][k]), int(iu[1][k])) for k in order[:4]}
    planted = {(int(p[0]), int(p[1])) for p in s.pairs}
    assert len(top & planted) >= 3
