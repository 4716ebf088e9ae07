"""Order-independent 64-bit digest of a row's coupled pairs (test helper).

A row's digest is the sum, modulo 2^64, of mix(j << 32 | g) over its pairs
(j: coupled sample, g: group id of x_i ^ x_j), with mix the 64-bit finaliser
of splitmix64 (S. Vigna; G. Steele, D. Lea, C. Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014).  Any reordering of a row's
pairs gives the same digest; a missing, extra or changed pair changes it
except with probability about 2^-64.  Both sides of a comparison compute it
here, from (i, j, g) arrays.
"""
from __future__ import annotations

import numpy as np

_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def mix64(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= _M1
        z ^= z >> np.uint64(27)
        z *= _M2
        z ^= z >> np.uint64(31)
    return z


def row_digests(i: np.ndarray, j: np.ndarray, g: np.ndarray, rows: np.ndarray):
    """(count, digest) of every row in `rows` (sorted ascending, unique) from
    pairs (i, j, g); pairs of other rows are ignored."""
    rows = np.asarray(rows, dtype=np.int64)
    i = np.asarray(i, dtype=np.int64)
    pos = np.searchsorted(rows, i)
    inside = (pos < rows.size) & (rows[np.minimum(pos, rows.size - 1)] == i)
    pos = pos[inside]
    v = mix64((np.asarray(j, dtype=np.uint64)[inside] << np.uint64(32)) |
              np.asarray(g, dtype=np.uint64)[inside])
    count = np.bincount(pos, minlength=rows.size).astype(np.int64)
    dig = np.zeros(rows.size, dtype=np.uint64)
    with np.errstate(over="ignore"):
        np.add.at(dig, pos, v)
    return count, dig
