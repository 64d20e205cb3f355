"""Residue alphabet, sequence encoding and the substitution-matrix loader.

This module turns amino-acid strings into the padded byte rows that every stage of the
path consumes, and loads the substitution matrix that the alignment stage takes as an
input. It contains none of the method's arithmetic.

Encoding (the paper's preprocessing trims/pads sequences, Sec. 3.5 and Algorithm 1,
preprocessing step; it fixes neither an alphabet order nor a pad value, so these are our
reading):
  * the 20 standard amino acids, coded 0..19 in the one-letter order ``ACDEFGHIKLMNPQRSTVWY``;
  * every sequence is stored in a row of ``stride`` bytes, positions past its length hold
    ``PAD`` (0xFF);
  * any other letter is rejected.
"""
from __future__ import annotations

import os

import numpy as np

ALPHABET = "ACDEFGHIKLMNPQRSTVWY"
PAD = 0xFF
_CODE = {c: i for i, c in enumerate(ALPHABET)}

_HERE = os.path.dirname(os.path.abspath(__file__))
BLOSUM62_PATH = os.path.join(_HERE, "blosum62.txt")


def encode(strings, stride: int = 32):
    """Encode amino-acid strings into ``(uint8[n][stride], int32[n])``.

    Raises ``ValueError`` for a letter outside the alphabet or a string longer than
    ``stride``.
    """
    n = len(strings)
    seqs = np.full((n, stride), PAD, dtype=np.uint8)
    lens = np.zeros(n, dtype=np.int32)
    for i, s in enumerate(strings):
        if len(s) > stride:
            raise ValueError(f"sequence {i} has length {len(s)} > stride {stride}")
        try:
            seqs[i, : len(s)] = [_CODE[c] for c in s]
        except KeyError as exc:
            raise ValueError(f"sequence {i} holds a non-standard residue {exc}") from None
        lens[i] = len(s)
    return seqs, lens


def decode(row, length: int) -> str:
    """Inverse of :func:`encode` for one row."""
    return "".join(ALPHABET[int(c)] for c in row[:length])


def load_blosum62(path: str = BLOSUM62_PATH) -> np.ndarray:
    """Load BLOSUM62 as ``int8[20][20]`` indexed in ``ALPHABET`` order.

    The file lists rows and columns in its own letter order; entries are placed by letter.
    """
    rows = []
    header = None
    with open(path) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            tok = line.split()
            if header is None:
                header = tok
                continue
            rows.append((tok[0], [int(v) for v in tok[1:]]))
    if header is None or len(rows) != len(header):
        raise ValueError("malformed substitution matrix file")
    out = np.zeros((20, 20), dtype=np.int8)
    seen = set()
    for letter, vals in rows:
        if len(vals) != len(header):
            raise ValueError(f"row {letter} has {len(vals)} entries")
        for col_letter, v in zip(header, vals):
            out[_CODE[letter], _CODE[col_letter]] = v
        seen.add(letter)
    if seen != set(ALPHABET) or set(header) != set(ALPHABET):
        raise ValueError("substitution matrix does not cover exactly the 20 residues")
    return out
