"""Write ``closed_forms.tsv``: pair cases whose answer is fixed by exact
rational arithmetic, with no call to either implementation.

Citation: the predicate is that of the "Sky" functional case (paper Section
2.1): B matches A when its distance from A is within the limits of the area
(circle, or ellipse with semi-axes and a position angle with zero-point and
direction of rotation), boundary inclusive (a reading; the paper is silent).

Each row is one (A, B, area) case. The coordinates are chosen so the exact
great-circle angle is a rational function of the inputs:

* meridian   RA_A = RA_B:            theta = |Dec_B - Dec_A|
* equator    Dec_A = Dec_B = 0:      theta = min(|dRA|, 360 - |dRA|)
* pole       RA_B = RA_A + 180:      theta = (90 - Dec_A) + (90 - Dec_B)
* ellipse    A on the equator, B due N/S (same RA) or due E/W (Dec 0):
             bearing 0/180/90/270 exactly, and with T in {0, 90, 180, 270}
             B lies on an axis, so inside <=> theta <= a (major) or b (minor).

B is placed 0..4 ulps either side of the boundary, so most cases sit inside
the FP64 uncertainty band and exercise the exact fallback.

Run: python tests/golden/make_closed_forms.py  (rewrites the .tsv)
"""
from __future__ import annotations

import math
import os
from fractions import Fraction as F

import numpy as np

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "closed_forms.tsv")


def ulps(x: float, k: int) -> float:
    d = math.inf if k > 0 else -math.inf
    for _ in range(abs(k)):
        x = math.nextafter(x, d)
    return x


def rows():
    out = []
    rng = np.random.default_rng(20161127)
    # --- meridian --------------------------------------------------------------
    for r in (1.0, 2.0, 0.5, 7.25, 225.0, 3600.0):
        for _ in range(6):
            ra = float(rng.uniform(0, 360))
            dec = float(rng.uniform(-85, 85))
            base = dec + r / 3600.0
            for k in range(-4, 5):
                decb = ulps(base, k)
                theta = abs(F(decb) - F(dec))
                inside = theta <= F(r) / 3600
                out.append(("meridian", ra, dec, ra, decb, 0, r, 0, 0, 0, 0, 1, int(inside)))
    # --- equator with and without the RA wrap ---------------------------------
    for r in (1.0, 2.0, 0.72, 36.0):
        for ra_a in (359.9998, 0.0001, 180.0, 359.99999999, 0.0, 123.456):
            for sgn in (1, -1):
                base = ra_a + sgn * r / 3600.0
                if base >= 360.0:
                    base -= 360.0
                if base < 0.0:
                    base += 360.0
                for k in range(-3, 4):
                    rab = ulps(base, k)
                    if not (0.0 <= rab < 360.0):
                        continue
                    d = abs(F(rab) - F(ra_a))
                    theta = min(d, 360 - d)
                    inside = theta <= F(r) / 3600
                    out.append(("equator", ra_a, 0.0, rab, 0.0, 0, r, 0, 0, 0, 0, 1, int(inside)))
    # --- through the pole -------------------------------------------------------
    for r in (1.0, 2.0, 10.0):
        for hemi in (1, -1):
            for ra_a in (0.0, 45.0, 200.0):
                ra_b = ra_a + 180.0 if ra_a < 180.0 else ra_a - 180.0
                base = hemi * (90.0 - r / 7200.0)
                for k in range(-3, 4):
                    d = ulps(base, k)
                    if abs(d) > 90.0:
                        continue
                    theta = 2 * (90 - abs(F(d)))
                    inside = theta <= F(r) / 3600
                    out.append(("pole", ra_a, d, ra_b, d, 0, r, 0, 0, 0, 0, 1, int(inside)))
                # unequal latitudes
                d1 = hemi * (90.0 - r / 3600.0 * 0.25)
                base2 = hemi * (90.0 - (r / 3600.0 - (90.0 - abs(d1))))
                for k in range(-3, 4):
                    d2 = ulps(base2, k)
                    if abs(d2) > 90.0:
                        continue
                    theta = (90 - abs(F(d1))) + (90 - abs(F(d2)))
                    inside = theta <= F(r) / 3600
                    out.append(("pole2", ra_a, d1, ra_b, d2, 0, r, 0, 0, 0, 0, 1, int(inside)))
    # --- ellipse on its axes ---------------------------------------------------
    combos = [  # (pa_zero, sense, pa) -> T = pa_zero + sense * pa
        (0.0, 1, 0.0), (0.0, 1, 90.0), (90.0, -1, 0.0), (180.0, -1, 90.0),
        (0.0, -1, 90.0), (270.0, 1, 0.0), (45.0, 1, 45.0), (90.0, 1, 90.0),
    ]
    for a, b in ((20.0, 10.0), (7.5, 2.25), (60.0, 18.0), (5.0, 5.0)):
        for pz, sense, pa in combos:
            T = (pz + sense * pa) % 360.0
            for ra_a in (10.0, 359.99999, 0.000001):
                for bearing in (0, 90, 180, 270):
                    along_major = ((bearing - T) % 180.0) == 0.0
                    lim = a if along_major else b
                    for k in range(-2, 3):
                        t = ulps(lim / 3600.0, k)
                        if bearing == 0:
                            rb, db = ra_a, t
                        elif bearing == 180:
                            rb, db = ra_a, -t
                        elif bearing == 90:
                            rb, db = ra_a + t, 0.0
                        else:
                            rb, db = ra_a - t, 0.0
                        if rb >= 360.0:
                            rb -= 360.0
                        if rb < 0.0:
                            rb += 360.0
                        if bearing in (90, 270):
                            d = abs(F(rb) - F(ra_a))
                            theta = min(d, 360 - d)
                        else:
                            theta = abs(F(db))
                        inside = theta <= F(lim) / 3600
                        out.append(("ellipse_axis", ra_a, 0.0, rb, db, 1, 0.0, a, b, pa, pz, sense,
                                    int(inside)))
    return out


HEADER = ("# kind\traA\tdecA\traB\tdecB\tshape\tradius_arcsec\ta_arcsec\tb_arcsec\tpa_deg"
          "\tpa_zero_deg\tpa_sense\tinside\n")


def main():
    with open(OUT, "w") as f:
        f.write("# Closed-form cross-match cases; exact answers from rational arithmetic.\n")
        f.write("# Predicate: paper Section 2.1 (Sky case), boundary inclusive.\n")
        f.write("# Written by make_closed_forms.py; floats are Python repr (round-trip exact).\n")
        f.write(HEADER)
        for r in rows():
            f.write("\t".join(repr(v) if isinstance(v, float) else str(v) for v in r) + "\n")


if __name__ == "__main__":
    main()
