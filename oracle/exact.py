"""Extended-precision decider for the cross-match oracle (mpmath, 200 bits).

TEST INFRASTRUCTURE: used only by the oracle package (tests, the smoke check
and the benchmark's CPU baseline). The GPU library never imports it.

The exact predicates of the paper's "Sky" case (Section 2.1) on inputs taken
as exact reals:

* circle : theta <= r
* ellipse: (theta/sin theta)^2 [(su/a)^2 + (sv/b)^2] <= 1, with (su, sv) the
  tangent-plane components of B seen from A rotated by T = pa_zero +
  pa_sense * PA (north towards east). a = b reduces to theta <= a.
* rectangle: (theta/sin theta) |su| <= a and (theta/sin theta) |sv| <= b
  (half-sides a along T, b across).
* best   : argmin over the matches of (theta, j), exact; an exact tie goes to
  the lower j (Section 2.2 keeps "only the best pairs"; the tie rule is the
  reading taken here).

At 200 bits every value is known to ~1e-58 relative; a difference from the
threshold below 1e-45 relative is treated as an exact tie, which the
inclusive boundary puts inside.
"""
from __future__ import annotations

from typing import Iterable, List, Optional, Sequence, Tuple

import math

import mpmath
from mpmath import mp, mpf

PREC_BITS = 200
TIE_REL = mpf("1e-45")


class _prec:
    def __enter__(self):
        self._old = mp.prec
        mp.prec = PREC_BITS
        return self

    def __exit__(self, *exc):
        mp.prec = self._old
        return False


def _k():
    return mp.pi / 180


def _pieces(ra1, dec1, ra2, dec2):
    k = _k()
    d1 = mpf(float(dec1)) * k
    d2 = mpf(float(dec2)) * k
    dd = (mpf(float(dec2)) - mpf(float(dec1))) * k
    da = (mpf(float(ra2)) - mpf(float(ra1))) * k
    return d1, d2, dd, da


def theta(ra1: float, dec1: float, ra2: float, dec2: float) -> mpf:
    """Great-circle angle (radians) between two points given in degrees."""
    with _prec():
        d1, d2, dd, da = _pieces(ra1, dec1, ra2, dec2)
        h = mpmath.sin(dd / 2) ** 2 + mpmath.cos(d1) * mpmath.cos(d2) * mpmath.sin(da / 2) ** 2
        if h < 0:
            h = mpf(0)
        return 2 * mpmath.asin(mpmath.sqrt(h))


def same_point(ra1, dec1, ra2, dec2) -> bool:
    return float(dec1) == float(dec2) and (float(ra1) == float(ra2) or abs(float(dec1)) == 90.0)


def decide_circle(ra1, dec1, ra2, dec2, r_arcsec) -> bool:
    """Exact theta <= r (r in arcsec), inclusive."""
    if float(r_arcsec) == 0.0:
        return same_point(ra1, dec1, ra2, dec2)
    with _prec():
        th = theta(ra1, dec1, ra2, dec2)
        R = mpf(float(r_arcsec)) / 3600 * _k()
        diff = th - R
        if abs(diff) <= TIE_REL * R:
            return True
        return diff < 0


def axis_xy(ra1, dec1, ra2, dec2, a_arcsec, b_arcsec, pa_deg, pa_zero_deg=0.0, pa_sense=1):
    """(u/a, v/b) at 200 bits: the azimuthal-equidistant coordinates of B seen
    from A (theta times the cosine and sine of the bearing from the axis T)
    over the semi-axes (half-sides); (0, 0) at theta = 0."""
    with _prec():
        k = _k()
        d1, d2, dd, da = _pieces(ra1, dec1, ra2, dec2)
        h = mpmath.sin(dd / 2) ** 2 + mpmath.cos(d1) * mpmath.cos(d2) * mpmath.sin(da / 2) ** 2
        if h <= 0:
            return mpf(0), mpf(0)
        th = 2 * mpmath.asin(mpmath.sqrt(h))
        tn = mpmath.sin(dd) + 2 * mpmath.sin(d1) * mpmath.cos(d2) * mpmath.sin(da / 2) ** 2
        te = mpmath.cos(d2) * mpmath.sin(da)
        T = (mpf(float(pa_zero_deg)) + int(pa_sense) * mpf(float(pa_deg))) * k
        su = tn * mpmath.cos(T) + te * mpmath.sin(T)
        sv = te * mpmath.cos(T) - tn * mpmath.sin(T)
        A = mpf(float(a_arcsec)) / 3600 * k
        B = mpf(float(b_arcsec)) / 3600 * k
        f = th / mpmath.sin(th)
        return f * su / A, f * sv / B


def decide_rect(ra1, dec1, ra2, dec2, a_arcsec, b_arcsec, pa_deg, pa_zero_deg=0.0,
                pa_sense=1) -> bool:
    """Rectangle of half-sides a (along T) and b (across): |u| <= a and
    |v| <= b, each boundary inclusive (a value within TIE_REL of it counts as
    on it)."""
    with _prec():
        x, y = axis_xy(ra1, dec1, ra2, dec2, a_arcsec, b_arcsec, pa_deg, pa_zero_deg, pa_sense)
        for t in (abs(x), abs(y)):
            if t > 1 and abs(t - 1) > TIE_REL:
                return False
        return True


def ellipse_q(ra1, dec1, ra2, dec2, a_arcsec, b_arcsec, pa_deg, pa_zero_deg=0.0, pa_sense=1):
    """The ellipse form Q (1 on the boundary) at 200 bits."""
    with _prec():
        k = _k()
        d1, d2, dd, da = _pieces(ra1, dec1, ra2, dec2)
        h = mpmath.sin(dd / 2) ** 2 + mpmath.cos(d1) * mpmath.cos(d2) * mpmath.sin(da / 2) ** 2
        if h <= 0:
            return mpf(0)
        th = 2 * mpmath.asin(mpmath.sqrt(h))
        tn = mpmath.sin(dd) + 2 * mpmath.sin(d1) * mpmath.cos(d2) * mpmath.sin(da / 2) ** 2
        te = mpmath.cos(d2) * mpmath.sin(da)
        T = (mpf(float(pa_zero_deg)) + int(pa_sense) * mpf(float(pa_deg))) * k
        su = tn * mpmath.cos(T) + te * mpmath.sin(T)
        sv = te * mpmath.cos(T) - tn * mpmath.sin(T)
        A = mpf(float(a_arcsec)) / 3600 * k
        B = mpf(float(b_arcsec)) / 3600 * k
        f = th / mpmath.sin(th)
        return f * f * ((su / A) ** 2 + (sv / B) ** 2)


def decide_ellipse(ra1, dec1, ra2, dec2, a_arcsec, b_arcsec, pa_deg, pa_zero_deg=0.0,
                   pa_sense=1) -> bool:
    with _prec():
        Q = ellipse_q(ra1, dec1, ra2, dec2, a_arcsec, b_arcsec, pa_deg, pa_zero_deg, pa_sense)
        if abs(Q - 1) <= TIE_REL:
            return True
        return Q < 1


def best_of(ra1, dec1, cand: Sequence[Tuple[int, float, float]]) -> int:
    """Exact argmin of (theta, j) over candidates (j, raB, decB)."""
    with _prec():
        best_j, best_t = None, None
        for j, rb, db in sorted(cand, key=lambda c: c[0]):
            t = theta(ra1, dec1, rb, db)
            if best_t is None:
                best_j, best_t = j, t
                continue
            tie = abs(t - best_t) <= TIE_REL * max(best_t, mpf("1e-300"))
            if not tie and t < best_t:
                best_j, best_t = j, t
        return int(best_j)


def brute(raA, decA, raB, decB, shape=0, radius_arcsec=1.0, a=None, b=None, pa=None,
          pa_zero_deg=0.0, pa_sense=1):
    """Brute-force exact join for tiny catalogues.

    Pairs are skipped only when a float64 haversine says theta exceeds twice
    the reach (a margin no rounding can cross). Returns (sorted list of
    (i, j), best list with -1 for unmatched rows)."""
    import numpy as np

    raA = np.asarray(raA, dtype=np.float64)
    decA = np.asarray(decA, dtype=np.float64)
    raB = np.asarray(raB, dtype=np.float64)
    decB = np.asarray(decB, dtype=np.float64)
    pairs: List[Tuple[int, int]] = []
    best: List[int] = []
    k = math.pi / 180
    for i in range(raA.shape[0]):
        if shape == 2:
            reach = math.hypot(a[i], b[i]) / 3600.0 * k
        else:
            reach = (a[i] if shape == 1 else radius_arcsec) / 3600.0 * k
        dd = (decB - decA[i]) * k
        da = (raB - raA[i]) * k
        h = np.sin(dd / 2) ** 2 + np.cos(decA[i] * k) * np.cos(decB * k) * np.sin(da / 2) ** 2
        lim = math.sin(min(reach, math.pi / 2)) ** 2   # hav(2 reach) >= sin^2(reach)
        cand = np.nonzero(h <= max(lim, 1e-300) * 1.0001 + 1e-300)[0]
        hits = []
        for j in cand.tolist():
            if shape == 1:
                ok = decide_ellipse(raA[i], decA[i], raB[j], decB[j], a[i], b[i], pa[i],
                                    pa_zero_deg, pa_sense)
            elif shape == 2:
                ok = decide_rect(raA[i], decA[i], raB[j], decB[j], a[i], b[i], pa[i],
                                 pa_zero_deg, pa_sense)
            else:
                ok = decide_circle(raA[i], decA[i], raB[j], decB[j], radius_arcsec)
            if ok:
                hits.append(j)
                pairs.append((i, j))
        if hits:
            best.append(best_of(raA[i], decA[i], [(j, raB[j], decB[j]) for j in hits]))
        else:
            best.append(-1)
    return pairs, best
