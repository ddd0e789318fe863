"""Symmetric best pairs of a cross-match (Section 2.2: the "best" match
selection keeps only the best pairs).

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use this module (see the package
docstring); it shares no code with the GPU library.

Reading (the paper does not define "best pair" further): besides each A
row's best match (the nearest B row in its area, exact ties to the lower B
row), a pair is a best pair in the symmetric sense when it is the best match
seen from both catalogues:

- best_b(j): the nearest A row among the A rows whose areas hold B row j
  (the exact argmin of (theta, i) over the stored matches of j; -1 if none);
- (i, j) is a symmetric best pair when best(i) = j and best_b(j) = i.

Each A row and each B row is in at most one symmetric best pair.
"""
from __future__ import annotations

import numpy as np

from . import exact

NEAR_REL = 2.0 ** -38  # FP64 separations closer than this are ranked at 200 bits


def best_of_b(raA, decA, raB, decB, ia, ib, sep, nB):
    """Nearest A row of every B row among its matches, -1 when it has none.
    FP64 separations order the candidates; those within NEAR_REL (relative)
    of a row's minimum are ranked exactly (exact.best_of: theta is symmetric,
    so the B row takes the place of the centre)."""
    ia = np.asarray(ia, dtype=np.int64)
    ib = np.asarray(ib, dtype=np.int64)
    sep = np.asarray(sep, dtype=np.float64)
    out = np.full(nB, -1, dtype=np.int32)
    if ia.size == 0:
        return out
    order = np.lexsort((ia, sep, ib))       # by B row, then separation, then A row
    sb, sa, ss = ib[order], ia[order], sep[order]
    first = np.ones(sb.shape[0], dtype=bool)
    first[1:] = sb[1:] != sb[:-1]
    rows = sb[first]
    out[rows] = sa[first]
    mins = np.zeros(nB)
    mins[rows] = ss[first]
    near = (ss <= mins[sb] * (1.0 + NEAR_REL) + 1e-300) & ~first
    for j in np.unique(sb[near]).tolist():
        sel = (ib == j) & (sep <= mins[j] * (1.0 + NEAR_REL) + 1e-300)
        cand = [(int(i), float(raA[i]), float(decA[i])) for i in ia[sel].tolist()]
        out[j] = exact.best_of(raB[j], decB[j], cand)
    return out


def mutual(raA, decA, raB, decB, ia, ib, sep, best_idx, nB):
    """Symmetric best pairs of a match result (canonical arrays ia, ib, sep
    and the per-A best matches): (pairs A rows, B rows, separations) in A
    order, and best_b for every B row."""
    bb = best_of_b(raA, decA, raB, decB, ia, ib, sep, nB)
    best_idx = np.asarray(best_idx)
    rows = np.nonzero(best_idx >= 0)[0]
    keep = rows[bb[best_idx[rows]] == rows]
    pj = best_idx[keep]
    # the pair's separation as stored
    ia = np.asarray(ia)
    ib = np.asarray(ib)
    pos = np.searchsorted(ia.astype(np.int64) * (1 << 32) + ib,
                          keep.astype(np.int64) * (1 << 32) + pj)
    return keep.astype(np.int32), pj.astype(np.int32), np.asarray(sep)[pos], bb
