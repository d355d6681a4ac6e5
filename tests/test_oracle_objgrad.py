"""Pins for the oracle's per-site objective and gradient (sec. 3.4 step 3,
eqs. g_regdef2, g_gradh2, g_gradJ2).  CPU only.

Each pin comes from outside the oracle: the closed form at the origin,
brute-force enumeration of the Potts model (eq. potts_model), the
regulariser identity of sec. 3.2, finite differences and exact invariants."""
import math

import numpy as np
import pytest

import oracle
from oracle import brute
from tests.helpers import random_params, weighted_frequencies


def _toy(seed=0, B=60, N=6, q=4):
    rng = np.random.default_rng(seed)
    msa = rng.integers(0, q, size=(B, N), dtype=np.uint8)
    w = rng.uniform(0.2, 1.0, size=B)
    return msa, w, float(np.sum(w))


def test_objective_at_origin_is_beff_log_q():
    msa, w, beff = _toy(1, q=21, N=7)
    q = 21
    for r in range(7):
        f = oracle.site_objgrad(msa, r, w, beff, np.zeros(q), np.zeros((7, q, q)), grad=False)
        assert f == pytest.approx(beff * math.log(q), rel=1e-13)


def test_gradient_at_origin_matches_frequencies():
    # at h = J = 0 every conditional is uniform (P = 1/q), so the gradient is
    # B_eff (1/q - f_r(s)) and B_eff (f_i(k)/q - f_ri(s,k)) (sec. 3.1 frequencies)
    msa, w, beff = _toy(2, B=80, N=5, q=5)
    q, N = 5, 5
    fi, fij = weighted_frequencies(msa, w, q)
    for r in range(N):
        f, gh, gJ = oracle.site_objgrad(msa, r, w, beff, np.zeros(q), np.zeros((N, q, q)))
        np.testing.assert_allclose(gh, beff * (1.0 / q - fi[r]), atol=1e-12)
        for i in range(N):
            if i == r:
                assert np.all(gJ[i] == 0.0)
                continue
            # gJ[i, k, s] = d f / d J_ri(s, k)
            expect = beff * (fi[i][:, None] / q - fij[r, i].T)
            np.testing.assert_allclose(gJ[i], expect, atol=1e-12)


@pytest.mark.parametrize("N", [3, 4])
def test_objective_matches_bruteforce_conditionals(N):
    # -sum_b w_b log P(sigma_r | rest) with P from the enumerated joint
    # distribution equals the data part of f_r; this fixes the energies, the
    # log-softmax and the index convention J_ri(l,k) = J_ir(k,l) of sec. 3.
    q = 3
    rng = np.random.default_rng(N)
    h, Jsym = brute.random_model(N, q, rng)
    msa = rng.integers(0, q, size=(25, N), dtype=np.uint8)
    w = rng.uniform(0.3, 1.0, size=25)
    beff = float(w.sum())
    for r in range(N):
        hr, Jr = brute.site_params(h, Jsym, r)
        f = oracle.site_objgrad(msa, r, w, beff, hr, Jr, lambda_h=0.0, lambda_J=0.0, grad=False)
        exact = 0.0
        for b in range(25):
            p = brute.conditional(msa[b], r, h, Jsym)
            exact -= w[b] * math.log(p[msa[b, r]])
        assert f == pytest.approx(exact, rel=1e-12)


def test_sum_of_site_objectives_is_pseudolikelihood_plus_l2():
    # sec. 3.2: with lambda'_J = lambda_J / 2 (sec. 3.4 step 1) and couplings
    # shared between the two sites of each pair, sum_r g_r^reg equals
    # l_pseudo + R_l2 (eq. l2reg); l_pseudo from the enumerated conditionals.
    N, q = 4, 3
    rng = np.random.default_rng(7)
    h, Jsym = brute.random_model(N, q, rng)
    msa = rng.integers(0, q, size=(30, N), dtype=np.uint8)
    w = rng.uniform(0.3, 1.0, size=30)
    beff = float(w.sum())
    lh, lJ = 0.03, 0.07
    total = 0.0
    for r in range(N):
        hr, Jr = brute.site_params(h, Jsym, r)
        total += oracle.site_objgrad(msa, r, w, beff, hr, Jr, lh, lJ, grad=False) / beff
    lpseudo = 0.0
    for r in range(N):
        for b in range(30):
            p = brute.conditional(msa[b], r, h, Jsym)
            lpseudo -= w[b] * math.log(p[msa[b, r]]) / beff
    Rl2 = lh * np.sum(h ** 2) + lJ * sum(np.sum(Jsym[i, j] ** 2) for i in range(N) for j in range(i + 1, N))
    assert total == pytest.approx(lpseudo + Rl2, rel=1e-12)


def test_gradient_matches_central_differences():
    msa, w, beff = _toy(3, B=50, N=6, q=4)
    N, q = 6, 4
    h, J = random_params(4, N, q, 0.3, 0.3)
    rng = np.random.default_rng(5)
    lh, lJ = 0.01, 0.02
    for r in (0, 3, 5):
        hr, Jr = h[r].copy(), J[r].copy()
        f, gh, gJ = oracle.site_objgrad(msa, r, w, beff, hr, Jr, lh, lJ)
        eps = 1e-5
        for _ in range(12):
            which = rng.integers(0, 2)
            if which == 0:
                s = rng.integers(0, q)
                hp, hm = hr.copy(), hr.copy()
                hp[s] += eps
                hm[s] -= eps
                fd = (oracle.site_objgrad(msa, r, w, beff, hp, Jr, lh, lJ, grad=False)
                      - oracle.site_objgrad(msa, r, w, beff, hm, Jr, lh, lJ, grad=False)) / (2 * eps)
                assert gh[s] == pytest.approx(fd, abs=1e-6 * beff)
            else:
                i = rng.integers(0, N)
                k, s = rng.integers(0, q, size=2)
                Jp, Jm = Jr.copy(), Jr.copy()
                Jp[i, k, s] += eps
                Jm[i, k, s] -= eps
                fd = (oracle.site_objgrad(msa, r, w, beff, hr, Jp, lh, lJ, grad=False)
                      - oracle.site_objgrad(msa, r, w, beff, hr, Jm, lh, lJ, grad=False)) / (2 * eps)
                assert gJ[i, k, s] == pytest.approx(fd, abs=1e-6 * beff)


def test_self_block_is_ignored():
    msa, w, beff = _toy(6, N=5, q=4)
    h, J = random_params(7, 5, 4)
    r = 2
    J2 = J[r].copy()
    J2[r] = 5.0  # garbage in the self block
    a = oracle.site_objgrad(msa, r, w, beff, h[r], J[r], 0.01, 0.01)
    b = oracle.site_objgrad(msa, r, w, beff, h[r], J2, 0.01, 0.01)
    assert a[0] == b[0]
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    assert np.all(b[2][r] == 0.0)


def test_data_gradient_sum_invariants():
    # with the regulariser off: sum_s dh(s) = 0; sum_s dJ_ri(s,k) = 0 for each k;
    # sum_k dJ_ri(s,k) = dh(s) for each i != r (every sequence has one state at i)
    msa, w, beff = _toy(8, B=70, N=6, q=5)
    h, J = random_params(9, 6, 5, 0.5, 0.5)
    for r in range(6):
        f, gh, gJ = oracle.site_objgrad(msa, r, w, beff, h[r], J[r], 0.0, 0.0)
        assert abs(gh.sum()) < 1e-12 * beff
        for i in range(6):
            if i == r:
                continue
            np.testing.assert_allclose(gJ[i].sum(axis=1), 0.0, atol=1e-12 * beff)
            np.testing.assert_allclose(gJ[i].sum(axis=0), gh, atol=1e-12 * beff)


def test_multi_site_wrapper_matches_single_site():
    msa, w, beff = _toy(10, B=40, N=5, q=4)
    h, J = random_params(11, 5, 4)
    f, gh, gJ = oracle.objgrad(msa, w, beff, h, J, 0.01, 0.02, sites=[4, 1], nthreads=2)
    for t, r in enumerate([4, 1]):
        f1, gh1, gJ1 = oracle.site_objgrad(msa, r, w, beff, h[r], J[r], 0.01, 0.02)
        assert f[t] == f1 and np.array_equal(gh[t], gh1) and np.array_equal(gJ[t], gJ1)


def test_slice_wrapper_matches_full_arrays():
    msa, w, beff = _toy(12, B=30, N=6, q=4)
    h, J = random_params(13, 6, 4)
    sites = [5, 0, 2]
    f, gh, gJ = oracle.objgrad(msa, w, beff, h, J, 0.01, 0.03, sites=sites)
    f2, gh2, gJ2 = oracle.objgrad_slices(msa, w, beff, h[sites], J[sites], sites, 0.01, 0.03, nthreads=3)
    assert np.array_equal(f, f2) and np.array_equal(gh, gh2) and np.array_equal(gJ, gJ2)
