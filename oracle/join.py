"""Join types of a cross-match (Section 2.2, "Match selection and join types").

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use this module (see the package
docstring); it shares no code with the GPU library.

The paper stores a cross-match as rows and offers five ways to combine the
matched and the unmatched rows of the two catalogues (catalogue 1 = A,
catalogue 2 = B):

- ``1and2``: only the matched rows (the stored pairs);
- ``1or2``: every row of both catalogues, matched or not;
- ``all1`` (``all2``): the matched rows plus the unmatched rows of catalogue
  1 (of catalogue 2);
- ``1not2`` (``2not1``): the rows of catalogue 1 (2) that have no match;
- ``1xor2``: only the unmatched rows of both catalogues.

Each is a union of three sets, written out here from those definitions: the
stored pairs, the unmatched A rows (no stored pair has them), and the
unmatched B rows (no stored pair has them). The stored pairs are all the
matches, or only each A row's best pair (the paper's two match selections).

Reading (the paper does not say): under the best selection a B row counts as
matched when it is the best match of some A row, i.e. when it appears in a
stored pair; an A row is matched under either selection exactly when it has
at least one match.
"""
from __future__ import annotations

import numpy as np

JOINS = ("1and2", "1or2", "all1", "all2", "1not2", "2not1", "1xor2")

# join -> (stored pairs, unmatched A rows, unmatched B rows)
PARTS = {
    "1and2": (True, False, False),
    "1or2": (True, True, True),
    "all1": (True, True, False),
    "all2": (True, False, True),
    "1not2": (False, True, False),
    "2not1": (False, False, True),
    "1xor2": (False, True, True),
}


def stored_pairs(ia, ib, best_idx, selection):
    """The stored pairs of a match result: every match (selection "all", the
    canonical (ia, ib) arrays) or each matched A row with its best match
    (selection "best", in A order)."""
    if selection == "all":
        return np.asarray(ia, dtype=np.int32), np.asarray(ib, dtype=np.int32)
    if selection == "best":
        best_idx = np.asarray(best_idx)
        rows = np.nonzero(best_idx >= 0)[0]
        return rows.astype(np.int32), best_idx[rows].astype(np.int32)
    raise ValueError("selection must be 'all' or 'best'")


def unmatched(nA, nB, pa, pb):
    """Rows of each catalogue that appear in no stored pair, ascending."""
    inA = np.zeros(nA, dtype=bool)
    inB = np.zeros(nB, dtype=bool)
    inA[np.asarray(pa, dtype=np.int64)] = True
    inB[np.asarray(pb, dtype=np.int64)] = True
    return (np.nonzero(~inA)[0].astype(np.int32), np.nonzero(~inB)[0].astype(np.int32))


def join(nA, nB, pa, pb, how):
    """The rows of join type ``how`` as four arrays: the stored pairs it keeps
    (A rows, B rows) and the unmatched A and B rows it keeps; parts a join
    leaves out are empty."""
    if how not in PARTS:
        raise ValueError(f"join must be one of {JOINS}")
    keep_p, keep_a, keep_b = PARTS[how]
    ua, ub = unmatched(nA, nB, pa, pb)
    empty = np.zeros(0, dtype=np.int32)
    return (np.asarray(pa, dtype=np.int32) if keep_p else empty,
            np.asarray(pb, dtype=np.int32) if keep_p else empty,
            ua if keep_a else empty,
            ub if keep_b else empty)
