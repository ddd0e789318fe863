"""Concentric ellipses of ClumpPopulator (Section 3, "A C^3 customized
version: ClumpPopulator").

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use this module (see the package
docstring); it shares no code with the GPU library.

ClumpPopulator extends the elliptical association to further ellipses
concentric with each source's own, scaled up or down. Written out from that
description, with these readings (the paper gives no formula):

- scale factors k_0 < k_1 < ... < k_{M-1} (> 0) are common to all sources;
  ellipse m of a source has semi-axes a * k_m and b * k_m, each product
  rounded to FP64 (the scaled axes are the doubles a * k_m, b * k_m), and
  the source's centre and position angle;
- the stored pairs are those of the largest ellipse (k_{M-1});
- each pair carries its level: the smallest m whose ellipse contains the B
  source (the ellipses are nested, so every larger one contains it too).

Each ellipse is decided by the certified ``oracle.match`` (Section 2.1,
"Sky" case, elliptical area).
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Concentric:
    ia: np.ndarray     # int32, canonical (ia, ib) order: pairs of the largest ellipse
    ib: np.ndarray     # int32
    sep: np.ndarray    # float64 arcsec
    level: np.ndarray  # int32: smallest scale index whose ellipse holds the pair


def check_scales(scales):
    k = np.asarray(scales, dtype=np.float64)
    if k.ndim != 1 or k.size == 0:
        raise ValueError("scales: a non-empty list")
    if not (np.all(np.isfinite(k)) and np.all(k > 0.0) and np.all(np.diff(k) > 0.0)):
        raise ValueError("scales must be finite, positive and strictly increasing")
    return k


def concentric(raA, decA, raB, decB, a, b, pa, scales, pa_zero_deg=0.0, pa_sense=1,
               nthreads=None) -> Concentric:
    """Pairs of the largest ellipse and their levels (one certified ellipse
    match per scale)."""
    import oracle
    k = check_scales(scales)
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    runs = []
    for km in k:
        runs.append(oracle.match(raA, decA, raB, decB, shape=1, a=a * km, b=b * km, pa=pa,
                                 pa_zero_deg=pa_zero_deg, pa_sense=pa_sense, nthreads=nthreads))
    outer = runs[-1]
    key = outer.ia.astype(np.int64) * (1 << 31) + outer.ib
    level = np.full(key.size, k.size - 1, dtype=np.int32)
    for m in range(k.size - 2, -1, -1):
        km_key = runs[m].ia.astype(np.int64) * (1 << 31) + runs[m].ib
        pos = np.searchsorted(key, km_key)
        if km_key.size and not (np.all(pos < key.size) and np.array_equal(key[pos], km_key)):
            raise AssertionError("ellipses are not nested")
        level[pos] = m
    return Concentric(outer.ia, outer.ib, outer.sep, level)


def levels_brute(raA, decA, raB, decB, a, b, pa, scales, pa_zero_deg=0.0, pa_sense=1):
    """The same at 200 bits, pair by pair (tiny inputs): for every (A, B),
    the smallest m whose ellipse holds B, or none."""
    from oracle import exact
    k = check_scales(scales)
    out = []
    for i in range(len(raA)):
        for j in range(len(raB)):
            for m, km in enumerate(k):
                if exact.decide_ellipse(raA[i], decA[i], raB[j], decB[j], float(a[i] * km),
                                        float(b[i] * km), pa[i], pa_zero_deg, pa_sense):
                    out.append((i, j, m))
                    break
    return out
