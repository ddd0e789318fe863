"""Pins for the oracle's rectangular region (paper Section 2.1 names an
elliptical, circular or rectangular region centred on the A source; here
|u| <= a and |v| <= b in the same azimuthal-equidistant frame as the
ellipse, a along the orientation T, b across):

* the closed-form axis rows of tests/golden/closed_forms.tsv: B on an axis of
  the area, where the rectangle and the ellipse agree exactly (inside iff
  theta <= a along T, theta <= b across), decided from rational arithmetic;
* corners and edge points placed by an independent 200-bit destination
  formula at (1 -+ 1e-9) of their exact distance, at several latitudes and
  orientations: inside, then outside;
* 200-bit brute force (oracle/exact.py) on small random catalogues, zones
  and brute force;
* invariants: ellipse(a, b) within rectangle(a, b) within circle(hypot(a,
  b)); T and T + 180 give the same set; Dec mirror.
"""
import math

import numpy as np
import pytest

import synth
from test_oracle_pins import CLOSED, _dest_mp


def test_axis_closed_forms(oracle_lib):
    rows = [r for r in CLOSED if r["kind"] == "ellipse_axis"]
    assert len(rows) > 1000
    wrong = [r for r in rows
             if oracle_lib.decide_exact(r["raA"], r["decA"], r["raB"], r["decB"], 2, 0.0, r["a"],
                                        r["b"], r["pa"], r["pz"], r["sense"]) != r["inside"]]
    assert not wrong, wrong[:3]
    n_amb = sum(oracle_lib.decide(r["raA"], r["decA"], r["raB"], r["decB"], 2, 0.0, r["a"], r["b"],
                                  r["pa"], r["pz"], r["sense"]) == 2 for r in rows)
    assert n_amb > len(rows) // 4  # ulp-adjacent rows reach the 200-bit decider


def _placements():
    """(dec, pz, sense, pa, a, b, bearing, dist_deg, inside) for corners and
    edge points of rectangles at known orientation."""
    out = []
    for dec in (0.0, 41.0, -72.5, 89.0):
        for (pz, sense, pa) in ((0.0, 1, 30.0), (90.0, -1, 12.5), (-15.0, 1, 100.0)):
            a, b = 24.0, 9.0
            T = pz + sense * pa
            pts = [(a, b), (-a, b), (a, -b), (-a, -b),          # corners
                   (a, 0.4 * b), (-0.3 * a, b), (0.9 * a, -b)]  # edges
            for u, v in pts:
                psi = math.degrees(math.atan2(v, u))
                dist = math.hypot(u, v) / 3600.0
                for f, want in ((1 - 1e-9, True), (1 + 1e-9, False)):
                    out.append((dec, pz, sense, pa, a, b, T + psi, dist * f, want))
    return out


@pytest.mark.parametrize("method", ["decide", "zones"])
def test_corners_and_edges_at_known_orientation(oracle_lib, method):
    for dec, pz, sense, pa, a, b, brg, dist, want in _placements():
        rb, db = _dest_mp(47.0, dec, brg, dist)
        if method == "decide":
            got = oracle_lib.decide_exact(47.0, dec, rb, db, 2, 0.0, a, b, pa, pz, sense)
            # 1e-9 from the boundary is far outside the FP64 margin: decided directly
            assert oracle_lib.decide(47.0, dec, rb, db, 2, 0.0, a, b, pa, pz, sense) == int(want)
        else:
            res = oracle_lib.match(np.array([47.0]), np.array([dec]), np.array([rb]),
                                   np.array([db]), shape=2, a=np.array([a]), b=np.array([b]),
                                   pa=np.array([pa]), pa_zero_deg=pz, pa_sense=sense)
            got = len(res.ia) == 1
        assert got == want, (dec, pz, sense, pa, brg, dist)


@pytest.mark.parametrize("lat", [(-89.0, 89.0), (88.0, 90.0), (-5.0, 5.0)])
def test_against_exact_brute_force(oracle_lib, lat):
    from test_oracle_pins import _near_boundary_catalogue
    raA, decA, raB, decB, a, b, pa = _near_boundary_catalogue(17, 40, 500, 1, lat=lat)
    # push B rows beyond the ellipse towards the corners: some rectangle-only pairs
    g = np.random.default_rng(18)
    par = g.integers(0, len(raA), 300)
    rb, db = synth.destination(raA[par], decA[par], g.uniform(0, 360, 300),
                               np.hypot(a[par], b[par]) * g.uniform(0.7, 1.05, 300) / 3600.0)
    raB, decB = np.concatenate([raB, rb]), np.concatenate([decB, db])
    kw = dict(a=a, b=b, pa=pa, pa_zero_deg=-40.0, pa_sense=1)
    pairs, best = oracle_lib.exact.brute(raA, decA, raB, decB, shape=2, **kw)
    for method in ("zones", "brute"):
        res = oracle_lib.match(raA, decA, raB, decB, shape=2, method=method, nthreads=2, **kw)
        assert list(zip(res.ia.tolist(), res.ib.tolist())) == sorted(pairs), method
        assert res.best_idx.tolist() == best
    ell = oracle_lib.match(raA, decA, raB, decB, shape=1, **kw)
    assert len(pairs) > len(ell.ia) + 20


def _pairs(res):
    return set(zip(res.ia.tolist(), res.ib.tolist()))


def test_invariants(oracle_lib):
    c = synth.cfg3_galactic_ellipses(scale=0.0004)
    kw = dict(a=c.a_arcsec, b=c.b_arcsec, pa=c.pa_deg, pa_sense=1)
    rect = _pairs(oracle_lib.match(c.raA, c.decA, c.raB, c.decB, shape=2, pa_zero_deg=20.0, **kw))
    ell = _pairs(oracle_lib.match(c.raA, c.decA, c.raB, c.decB, shape=1, pa_zero_deg=20.0, **kw))
    assert ell < rect and len(rect) > 100
    r180 = _pairs(oracle_lib.match(c.raA, c.decA, c.raB, c.decB, shape=2, pa_zero_deg=200.0,
                                   **kw))
    assert r180 == rect
    dm = _pairs(oracle_lib.match(c.raA, -c.decA, c.raB, -c.decB, shape=2, pa_zero_deg=160.0,
                                 a=c.a_arcsec, b=c.b_arcsec, pa=c.pa_deg, pa_sense=-1))
    assert dm == rect
    # every rectangle pair lies within the half-diagonal
    d = np.hypot(c.a_arcsec, c.b_arcsec)
    res = oracle_lib.match(c.raA, c.decA, c.raB, c.decB, shape=2, pa_zero_deg=20.0, **kw)
    assert np.all(res.sep <= d[res.ia] * (1 + 1e-12))
