"""Alignment ingestion through the C ABI (host code, no GPU) against the
oracle parser: the hand-worked fixtures, seeded random alignments written
as wrapped FASTA and interleaved Stockholm with inserts, and error cases."""
import os

import numpy as np
import pytest

from oracle import msa_io
from paper_1401_4832_amd import api
from paper_1401_4832_amd._lib import PlmError

GOLD = os.path.join(os.path.dirname(__file__), "golden")
LETTERS = "ACDEFGHIKLMNPQRSTVWY"


def test_fixtures_match_oracle():
    for name in ("msa_small.fasta", "msa_small.sto"):
        path = os.path.join(GOLD, name)
        with open(path) as fh:
            expect = msa_io.parse(fh.read())
        np.testing.assert_array_equal(api.read_alignment(path), expect)


def _random_alignment(seed, B, N):
    rng = np.random.default_rng(seed)
    rows, texts = [], []
    for b in range(B):
        chars = []
        for i in range(N):
            u = rng.random()
            chars.append("-" if u < 0.15 else "X" if u < 0.17 else LETTERS[rng.integers(20)])
            if rng.random() < 0.1:  # an insert after this column
                chars.append(rng.choice(list("acdefghiklmnpqrstvwy.")))
        texts.append("".join(chars))
    return texts


@pytest.mark.parametrize("seed,B,N", [(1, 5, 7), (2, 40, 33), (3, 1, 1), (4, 17, 150)])
def test_random_fasta_and_stockholm(seed, B, N):
    seqs = _random_alignment(seed, B, N)
    rng = np.random.default_rng(seed + 100)
    fasta = []
    for b, s in enumerate(seqs):
        fasta.append(f">s{b} description {b}")
        w = int(rng.integers(5, 60))
        fasta += [s[k:k + w] for k in range(0, len(s), w)]
    fasta_text = "\n".join(fasta) + "\n"
    sto = ["# STOCKHOLM 1.0", "#=GF ID random"]
    cut = sorted(set(int(x) for x in rng.integers(0, max(1, min(len(s) for s in seqs)), size=2)))
    bounds = [0] + cut + [None]
    for k in range(len(bounds) - 1):
        for b, s in enumerate(seqs):
            sto.append(f"s{b}   {s[bounds[k]:bounds[k + 1]]}")
        sto.append("#=GC RF xxx")
        sto.append("")
    sto.append("//")
    sto_text = "\n".join(sto) + "\n"
    for text in (fasta_text, sto_text):
        expect = msa_io.parse(text)
        got = api.parse_alignment(text)
        assert got.shape == (B, N)
        np.testing.assert_array_equal(got, expect)


@pytest.mark.parametrize("text", [">a\nAC\n>b\nACD\n", ">a\nA1C\n", "ACD\n", "", "# STOCKHOLM 1.0\n//\n",
                                  ">a\nac\n"])
def test_errors_are_reported(text):
    with pytest.raises(ValueError):
        msa_io.parse(text)
    with pytest.raises(PlmError):
        api.parse_alignment(text)
