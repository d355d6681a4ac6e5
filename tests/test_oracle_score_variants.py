"""Pins of the score-variant oracle (sec. 7 alternatives, sec. 6 TPR) against
closed forms, invariants and the independently pinned CFN oracle."""
import math

import numpy as np
import pytest

import oracle
from oracle import score_variants as sv


def _random_J(seed, N, q, scale=0.4):
    rng = np.random.default_rng(seed)
    J = scale * rng.standard_normal((N, N, q, q))
    for r in range(N):
        J[r, r] = 0.0
    return J


def test_frobenius_avg_apc_equal_the_cfn_oracle():
    J = _random_J(1, 9, 5)
    fn_o, cfn_o = oracle.score(J)
    raw = sv.raw_scores(J, "avg", "frob")
    np.testing.assert_allclose(raw, fn_o, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(sv.correct(raw, "apc"), cfn_o, rtol=1e-11, atol=1e-13)
    # p = 2 of the l_p family is the Frobenius norm
    np.testing.assert_allclose(sv.raw_scores(J, "avg", "lp", p=2.0), raw, rtol=1e-13)


def test_consistent_model_makes_min_max_avg_agree():
    rng = np.random.default_rng(2)
    N, q = 6, 4
    J = np.zeros((N, N, q, q))
    for i in range(N):
        for j in range(i + 1, N):
            M = rng.standard_normal((q, q))  # (state i, state j)
            J[i, j] = M.T                    # J[i][j][k][s]: s = state of i, k = state of j
            J[j, i] = M                      # J[j][i][k][s]: s = state of j, k = state of i
    a = sv.raw_scores(J, "avg")
    assert np.allclose(sv.raw_scores(J, "min"), a, rtol=1e-13)
    assert np.allclose(sv.raw_scores(J, "max"), a, rtol=1e-13)
    # and they differ once the two estimates disagree
    J2 = J.copy()
    J2[0, 1, 0, 0] += 0.3  # (a constant shift would be removed by the gauge)
    assert not np.allclose(sv.raw_scores(J2, "min")[0, 1], sv.raw_scores(J2, "max")[0, 1])


def test_lp_closed_forms_and_monotonicity():
    rng = np.random.default_rng(3)
    M = sv.ising_gauge(rng.standard_normal((5, 5)))
    assert math.isclose(sv.pair_norm(M, "lp", p=1.0), float(np.abs(M).sum()), rel_tol=1e-13)
    vals = [sv.pair_norm(M, "lp", p=p) for p in (1.0, 1.5, 2.0, 3.0, 8.0)]
    assert all(a >= b for a, b in zip(vals, vals[1:]))
    assert vals[-1] >= np.abs(M).max()


def test_burkoff_two_state_closed_form_and_nonnegativity():
    # q = 2, uniform frequencies, Ising-gauge couplings [[a, -a], [-a, a]]:
    # D = ln 2 + t ln t + (1 - t) ln(1 - t) with t = e^a / (e^a + e^-a)
    for a in (0.0, 0.3, -1.1, 2.5):
        M = np.array([[a, -a], [-a, a]])
        J = np.zeros((2, 2, 2, 2))
        J[0, 1] = M.T
        J[1, 0] = M
        f = np.full((2, 2), 0.5)
        D = sv.raw_scores(J, "avg", "burkoff", freq=f)[0, 1]
        t = math.exp(a) / (math.exp(a) + math.exp(-a))
        expect = math.log(2.0) + t * math.log(t) + (1 - t) * math.log(1 - t)
        assert math.isclose(D, expect, rel_tol=1e-12, abs_tol=1e-15), (a, D, expect)
    rng = np.random.default_rng(4)
    J = _random_J(4, 6, 5, scale=0.8)
    f = rng.dirichlet(np.ones(5), size=6)
    D = sv.raw_scores(J, "avg", "burkoff", freq=f)
    assert np.all(D >= -1e-15)                 # a KL divergence
    assert np.all(np.abs(sv.raw_scores(np.zeros_like(J), "avg", "burkoff", freq=f)) <= 1e-15)


def test_gap_excluded_norm():
    a = 0.7
    q = 3  # the gap is state 2
    Ms = [np.array([[a, -a, 0], [-a, a, 0], [0, 0, 0]]),   # no weight on the gap
          np.array([[0, 0, 0], [0, a, -a], [0, -a, a]])]   # weight on the gap row/column
    expect_full = [2 * a, 2 * a]
    expect_nogap = [2 * a, a]
    for M, ef, eg in zip(Ms, expect_full, expect_nogap):
        J = np.zeros((2, 2, q, q))
        J[0, 1] = M.T
        J[1, 0] = M
        assert math.isclose(sv.raw_scores(J)[0, 1], ef, rel_tol=1e-13)
        assert math.isclose(sv.raw_scores(J, exclude_gap=True)[0, 1], eg, rel_tol=1e-13)
    J = _random_J(5, 7, 6)
    assert np.all(sv.raw_scores(J, exclude_gap=True) <= sv.raw_scores(J) + 1e-15)


def test_average_sum_correction_row_sums():
    J = _random_J(6, 8, 4)
    S = sv.raw_scores(J)
    C = sv.correct(S, "asc")
    r, c, a = S.mean(axis=1), S.mean(axis=0), S.mean()
    # double centring, then the diagonal set to zero: row i sums to r_i + c_i - a
    np.testing.assert_allclose(C.sum(axis=1), r + c - a, rtol=1e-12, atol=1e-13)
    assert np.all(np.diag(C) == 0.0)
    np.testing.assert_array_equal(sv.correct(S, "none"), S)


def test_tpr_hand_worked():
    N = 8
    S = np.zeros((N, N))
    vals = {(0, 5): 0.9, (1, 7): 0.8, (0, 6): 0.7, (2, 7): 0.6, (0, 7): 0.5, (1, 6): 0.4,
            (0, 1): 5.0, (3, 4): 4.0}  # the last two are closer than 5 apart: ignored
    for (i, j), v in vals.items():
        S[i, j] = S[j, i] = v
    C = np.zeros((N, N), dtype=bool)
    for i, j in [(0, 5), (2, 7), (0, 1)]:
        C[i, j] = C[j, i] = True
    t = sv.tpr_curve(S, C, min_sep=5)
    np.testing.assert_allclose(t, [1, 1 / 2, 1 / 3, 2 / 4, 2 / 5, 2 / 6], rtol=1e-15)
    assert len(sv.tpr_curve(S, C, min_sep=5, kmax=3)) == 3


def test_frequencies_sum_to_one():
    rng = np.random.default_rng(7)
    msa = rng.integers(0, 6, size=(300, 9), dtype=np.uint8)
    w = rng.uniform(0.2, 1.0, size=300)
    f = sv.frequencies(msa, w, float(w.sum()), 6)
    np.testing.assert_allclose(f.sum(axis=1), 1.0, rtol=1e-13)
    f1 = sv.frequencies(msa, np.ones(300), 300.0, 6)
    np.testing.assert_allclose(f1[2], np.bincount(msa[:, 2], minlength=6) / 300.0, rtol=1e-15)
