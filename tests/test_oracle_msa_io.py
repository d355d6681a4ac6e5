"""Pins of the ingestion oracle: hand-worked fixtures (tests/golden, codes
derived by hand from the format rules) and the error cases."""
import os

import numpy as np
import pytest

from oracle import msa_io

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _expected():
    rows = []
    with open(os.path.join(GOLD, "msa_small_codes.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append([int(x) for x in line.split()])
    return np.array(rows[:3], dtype=np.uint8), np.array(rows[3:], dtype=np.uint8)


def test_fixtures():
    fa, sto = _expected()
    with open(os.path.join(GOLD, "msa_small.fasta")) as fh:
        np.testing.assert_array_equal(msa_io.parse(fh.read()), fa)
    with open(os.path.join(GOLD, "msa_small.sto")) as fh:
        np.testing.assert_array_equal(msa_io.parse(fh.read()), sto)


@pytest.mark.parametrize("text", [">a\nAC\n>b\nACD\n", ">a\nA1C\n", "ACD\n", "", "# STOCKHOLM 1.0\n//\n",
                                  ">a\nac\n"])
def test_errors(text):
    with pytest.raises(ValueError):
        msa_io.parse(text)
