"""Pins for the oracle's sequence reweighting (sec. 3.1, eq. inverse_weights;
sec. 3.4 step 2, eq. inverse_weights2).  CPU only."""
import os

import numpy as np
import pytest

import oracle
from tests.helpers import clustered_msa, load_reweight_golden

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "reweight_tiny.txt")


def test_hand_worked_example():
    rows, cases = load_reweight_golden(GOLDEN)
    for theta, m_expect in cases:
        m, w, beff = oracle.reweight(rows, theta=theta)
        assert m.tolist() == m_expect, theta
        assert np.array_equal(w, 1.0 / np.array(m_expect, dtype=np.float64))
        acc = 0.0
        for v in m_expect:
            acc += 1.0 / v
        assert beff == acc


def test_theta_zero_counts_everything():
    rng = np.random.default_rng(0)
    msa = rng.integers(0, 21, size=(37, 11), dtype=np.uint8)
    m, w, beff = oracle.reweight(msa, theta=0.0)
    assert np.all(m == 37)
    assert np.all(w == 1.0 / 37.0)
    acc = 0.0
    for _ in range(37):
        acc += 1.0 / 37.0
    assert beff == acc


def test_identical_rows():
    msa = np.tile(np.arange(9, dtype=np.uint8), (13, 1))
    for theta in (0.0, 0.5, 0.8, 1.0):
        m, w, beff = oracle.reweight(msa, theta=theta)
        assert np.all(m == 13)


def test_all_distinct_rows_have_unit_weight():
    # rows that pairwise agree in no column
    msa = np.array([[(a + i) % 21 for i in range(15)] for a in range(21)], dtype=np.uint8)
    m, w, beff = oracle.reweight(msa, theta=0.1)
    assert np.all(m == 1) and beff == 21.0


def test_theta_one_counts_exact_duplicates():
    rng = np.random.default_rng(3)
    base = rng.integers(0, 21, size=(10, 8), dtype=np.uint8)
    idx = rng.integers(0, 10, size=40)
    msa = base[idx]
    m, _, _ = oracle.reweight(msa, theta=1.0)
    for b in range(40):
        assert m[b] == int(np.sum(idx == idx[b])) or np.sum(np.all(msa == msa[b], axis=1)) == m[b]


def test_uniform_mode():
    msa = np.zeros((7, 3), dtype=np.uint8)
    m, w, beff = oracle.reweight(msa, theta=0.8, uniform=True)
    assert np.all(m == 1) and np.all(w == 1.0) and beff == 7.0


def test_rows_variant_and_symmetry():
    msa = clustered_msa(seed=11, B=300, N=40, n_anc=12, p_mut=0.12)
    m, _, _ = oracle.reweight(msa, theta=0.8)
    assert 1 < m.max() < 300  # non-trivial weights
    rows = np.array([0, 5, 17, 299, 123], dtype=np.int32)
    assert np.array_equal(oracle.reweight_rows(msa, rows, theta=0.8), m[rows])
    # similarity is symmetric: the number of similar ordered pairs is even
    # once the B self-pairs are removed
    assert (int(m.sum()) - 300) % 2 == 0


def test_threading_does_not_change_result():
    msa = clustered_msa(seed=5, B=200, N=30, n_anc=8, p_mut=0.15)
    a = oracle.reweight(msa, theta=0.8, nthreads=1)
    b = oracle.reweight(msa, theta=0.8, nthreads=7)
    assert np.array_equal(a[0], b[0]) and a[2] == b[2]
