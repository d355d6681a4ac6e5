"""The seeded input generator: determinism, shapes, ranges, planted structure."""
import numpy as np

import synth


def test_deterministic_and_in_range():
    a = synth.make_msa("t", N=20, B=130, npairs=10, seed=9, cache=False)
    b = synth.make_msa("t", N=20, B=130, npairs=10, seed=9, cache=False)
    assert a.msa.shape == (130, 20) and a.msa.dtype == np.uint8
    assert np.array_equal(a.msa, b.msa) and np.array_equal(a.pairs, b.pairs)
    assert a.msa.max() < 21
    c = synth.make_msa("t", N=20, B=130, npairs=10, seed=10, cache=False)
    assert not np.array_equal(a.msa, c.msa)


def test_planted_pairs_respect_separation_and_are_distinct():
    s = synth.make_msa("t", N=40, B=64, npairs=60, seed=3, min_sep=5, cache=False)
    p = s.pairs
    assert p.shape == (60, 2)
    assert np.all(p[:, 1] - p[:, 0] >= 5)
    assert len({tuple(x) for x in p}) == 60


def test_gap_forcing_rate():
    s = synth.make_msa("t", N=50, B=2000, npairs=10, seed=4, gap_p=0.1, cache=False)
    base = synth.make_msa("t", N=50, B=2000, npairs=10, seed=4, cache=False)
    forced = (s.msa == 20) & (base.msa != 20)
    rate = forced.sum() / (base.msa != 20).sum()
    assert 0.09 < rate < 0.11


def test_thread_count_does_not_matter(monkeypatch):
    a = synth.make_msa("t", N=15, B=200, npairs=5, seed=8, cache=False)
    monkeypatch.setattr(synth, "_threads", lambda: 1)
    b = synth.make_msa("t", N=15, B=200, npairs=5, seed=8, cache=False)
    assert np.array_equal(a.msa, b.msa)


def test_ragged_set_ranges():
    sets = synth.ragged_set(count=16, b_range=(200, 300), n_range=(60, 300), cache=False,
                            burnin=2, thin=1, nchains=4)
    assert len(sets) == 16
    for s in sets:
        assert 60 <= s.N <= 300 and 200 <= s.B <= 300
