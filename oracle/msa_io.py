"""Oracle of alignment ingestion (sec. 4): FASTA or Stockholm text to
symbol codes.  Test infrastructure only.

The paper's alignments come from PFAM, whose inserts (residues not aligned
to the model: lowercase letters, and "." in the other sequences) are removed
before DCA (sec. 4).  Readings: the 20 standard residues A C D E F G H I K L
M N P Q R S T V W Y are codes 0..19 in that order, "-" (gap) is code 20
(q = 21); the non-standard uppercase letters B J O U X Z count as gaps; "*"
(a sequence terminator in some FASTA files) is skipped; any other
character is an error, as are sequences of different aligned lengths.
Stockholm: "#" lines are annotation, "//" ends the alignment, every other
non-empty line is "name sequence-part", parts of one name concatenated in
order (interleaved blocks), sequences in order of first appearance.
"""
from __future__ import annotations

import numpy as np

ALPHABET = "ACDEFGHIKLMNPQRSTVWY"
GAP = 20
NONSTANDARD = "BJOUXZ"


def _codes(seq: str):
    out = []
    for ch in seq:
        if ch.islower() or ch == ".":
            continue  # insert
        if ch == "-":
            out.append(GAP)
        elif ch in ALPHABET:
            out.append(ALPHABET.index(ch))
        elif ch in NONSTANDARD:
            out.append(GAP)
        elif ch == "*":
            continue
        else:
            raise ValueError(f"unexpected character {ch!r}")
    return out


def parse(text: str, fmt: str = "auto") -> np.ndarray:
    lines = text.splitlines()
    if fmt == "auto":
        first = next((l for l in lines if l.strip()), "")
        fmt = "stockholm" if first.startswith("# STOCKHOLM") else "fasta" if first.lstrip().startswith(">") else None
        if fmt is None:
            raise ValueError("unknown alignment format")
    seqs = []
    if fmt == "fasta":
        cur = None
        for l in lines:
            if l.startswith(">"):
                cur = []
                seqs.append(cur)
            elif l.strip():
                if cur is None:
                    raise ValueError("sequence before the first header")
                cur.append("".join(l.split()))
        seqs = ["".join(s) for s in seqs]
    elif fmt == "stockholm":
        parts, order = {}, []
        for l in lines:
            t = l.strip()
            if not t or t.startswith("#"):
                continue
            if t == "//":
                break
            name, rest = t.split(None, 1) if len(t.split(None, 1)) == 2 else (t, "")
            if name not in parts:
                parts[name] = []
                order.append(name)
            parts[name].append("".join(rest.split()))
        seqs = ["".join(parts[n]) for n in order]
    else:
        raise ValueError(fmt)
    rows = [_codes(s) for s in seqs]
    if not rows:
        raise ValueError("no sequences")
    n = len(rows[0])
    if n == 0 or any(len(r) != n for r in rows):
        raise ValueError("sequences of different aligned lengths")
    return np.array(rows, dtype=np.uint8)
