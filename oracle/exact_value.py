"""The Exact Value functional case (Section 2.1: two rows match when the
values they hold in one chosen column each are equal), with the match
selections of Section 2.2.

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use this module (see the package
docstring); it shares no code with the GPU library.

Readings (the paper names the case and nothing more):

- the columns hold int64 or float64 values; equal means numerically equal
  (for float64, +0 equals -0 and a NaN equals nothing, itself included);
- "all": every pair (i, j) with vA[i] == vB[j], in (i, j) order;
- "best": every match of a row is equally good (the values are equal), so a
  row's best match is its first, the lowest B row;
- the join types are the Sky case's (oracle/join.py) applied to these pairs.

Written from the definition: a dictionary from each value to the ascending
list of B rows that hold it, looked up for every A row.
"""
from __future__ import annotations

import numpy as np


def _norm(v, kind):
    """Key of a value for the dictionary: the integer itself, or the float
    with -0 folded onto +0; None for a NaN (never equal)."""
    if kind == "i64":
        return int(v)
    x = float(v)
    if x != x:
        return None
    return 0.0 if x == 0.0 else x


def match(vA, vB, kind="i64"):
    """(ia, ib) of every match in canonical order, and best_idx per A row
    (-1 when unmatched)."""
    table = {}
    for j, v in enumerate(np.asarray(vB).tolist()):
        k = _norm(v, kind)
        if k is not None:
            table.setdefault(k, []).append(j)
    ia, ib = [], []
    best = np.full(len(vA), -1, dtype=np.int32)
    for i, v in enumerate(np.asarray(vA).tolist()):
        k = _norm(v, kind)
        rows = table.get(k) if k is not None else None
        if rows:
            best[i] = rows[0]
            ia.extend([i] * len(rows))
            ib.extend(rows)
    return np.asarray(ia, dtype=np.int32), np.asarray(ib, dtype=np.int32), best
