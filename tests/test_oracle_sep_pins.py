"""Pins of the oracle's separation (the distance of paper Section 2.1, the
angle between the central object and the B source), against values fixed
without the oracle's formula:

* closed forms: every row of tests/golden/closed_forms.tsv has an exact
  great-circle angle in rational arithmetic (same meridian: |dDec|; both on
  the equator: min(|dRA|, 360 - |dRA|); opposite meridians near a pole:
  (90 - |Dec_A|) + (90 - |Dec_B|));
* 200-bit values (oracle/exact.py theta, a haversine in mpmath) on random
  near-boundary catalogues, the polar caps included.

The separations the oracle reports (per pair and for the best match) must be
within 1e-9 arcsec of these, far inside the 1e-6 arcsec the GPU is held to.
"""
from fractions import Fraction as F

import numpy as np
import pytest

from test_oracle_pins import CLOSED, _near_boundary_catalogue

TOL = 1e-9  # arcsec


def exact_theta_deg(r) -> F:
    """Exact angle (degrees) of a closed-form row, from its geometry."""
    raA, decA, raB, decB = (F(r[k]) for k in ("raA", "decA", "raB", "decB"))
    if raA == raB:                          # one meridian
        return abs(decB - decA)
    if decA == 0 and decB == 0:             # the equator, wrap included
        d = abs(raB - raA)
        return min(d, 360 - d)
    d = abs(raB - raA)
    assert d == 180 and decA * decB > 0, r  # opposite meridians, one hemisphere
    return (90 - abs(decA)) + (90 - abs(decB))


EXACT = [float(exact_theta_deg(r) * 3600) for r in CLOSED]


def test_closed_form_geometry_covers_every_kind():
    kinds = {r["kind"] for r in CLOSED}
    assert kinds == {"meridian", "equator", "pole", "pole2", "ellipse_axis"}
    # angles span sub-arcsec to a degree
    assert min(EXACT) < 1.0 and max(EXACT) > 3000.0


def test_sep_closed_forms_every_row(oracle_lib):
    n = len(CLOSED)
    raA = np.array([r["raA"] for r in CLOSED])
    decA = np.array([r["decA"] for r in CLOSED])
    raB = np.array([r["raB"] for r in CLOSED])
    decB = np.array([r["decB"] for r in CLOSED])
    k = np.arange(n, dtype=np.int32)
    got = oracle_lib.seps(raA, decA, raB, decB, k, k)
    err = np.abs(got - np.array(EXACT))
    assert err.max() <= TOL, (err.argmax(), CLOSED[int(err.argmax())], got[err.argmax()])


def test_sep_closed_forms_through_join(oracle_lib):
    """Each closed-form pair inside its own join: the separation written for
    the diagonal pair, and the best match's separation, equal the exact
    angle."""
    groups = {}
    for idx, r in enumerate(CLOSED):
        groups.setdefault((r["shape"], r["r"], r["pz"], r["sense"]), []).append(idx)
    checked = 0
    for (shape, rad, pz, sense), ids in groups.items():
        rs = [CLOSED[i] for i in ids]
        raA = np.array([r["raA"] for r in rs])
        decA = np.array([r["decA"] for r in rs])
        raB = np.array([r["raB"] for r in rs])
        decB = np.array([r["decB"] for r in rs])
        kw = {}
        if shape == 1:
            kw = dict(a=np.array([r["a"] for r in rs]), b=np.array([r["b"] for r in rs]),
                      pa=np.array([r["pa"] for r in rs]), pa_zero_deg=pz, pa_sense=sense)
        res = oracle_lib.match(raA, decA, raB, decB, shape=shape, radius_arcsec=rad, nthreads=2,
                               **kw)
        for i, j, s in zip(res.ia.tolist(), res.ib.tolist(), res.sep.tolist()):
            want = float(exact_theta_deg(rs[j]) * 3600) if i == j else None
            if want is not None:
                assert abs(s - want) <= TOL, (rs[i], s, want)
                checked += 1
        for i in range(len(rs)):
            j = int(res.best_idx[i])
            if j < 0:
                continue
            want = float(exact_theta_deg({"raA": rs[i]["raA"], "decA": rs[i]["decA"],
                                          "raB": rs[j]["raB"], "decB": rs[j]["decB"]}) * 3600) \
                if _closed(rs[i], rs[j]) else None
            if want is not None:
                assert abs(res.best_sep[i] - want) <= TOL
    assert checked > 1000


def _closed(ra, rb):
    """Whether A of row ra and B of row rb still form a closed-form pair."""
    if ra["raA"] == rb["raB"]:
        return True
    if ra["decA"] == 0 and rb["decB"] == 0:
        return True
    d = abs(F(rb["raB"]) - F(ra["raA"]))
    return d == 180 and ra["decA"] * rb["decB"] > 0


@pytest.mark.parametrize("shape", [0, 1])
@pytest.mark.parametrize("lat", [(-89.0, 89.0), (88.0, 90.0), (-90.0, -88.0), (-1.0, 1.0)])
def test_sep_against_200_bit_theta(oracle_lib, shape, lat):
    raA, decA, raB, decB, a, b, pa = _near_boundary_catalogue(31 + shape, 60, 600, shape, lat=lat)
    kw = dict(a=a, b=b, pa=pa, pa_zero_deg=5.0, pa_sense=1) if shape == 1 else {}
    res = oracle_lib.match(raA, decA, raB, decB, shape=shape, radius_arcsec=2.0, nthreads=2, **kw)
    assert len(res.ia) > 100
    ex = oracle_lib.exact
    import mpmath
    conv = 180 * 3600 / mpmath.pi
    want = np.array([float(ex.theta(raA[i], decA[i], raB[j], decB[j]) * conv)
                     for i, j in zip(res.ia.tolist(), res.ib.tolist())])
    assert np.abs(res.sep - want).max() <= TOL
    rows = np.nonzero(res.best_idx >= 0)[0]
    wb = np.array([float(ex.theta(raA[i], decA[i], raB[res.best_idx[i]], decB[res.best_idx[i]])
                         * conv) for i in rows.tolist()])
    assert np.abs(res.best_sep[rows] - wb).max() <= TOL
    # every pair, matched or not, through the per-pair separation
    ia = np.repeat(np.arange(len(raA), dtype=np.int32), 4)
    ib = np.random.default_rng(5).integers(0, len(raB), ia.shape[0]).astype(np.int32)
    got = oracle_lib.seps(raA, decA, raB, decB, ia, ib)
    wa = np.array([float(ex.theta(raA[i], decA[i], raB[j], decB[j]) * conv)
                   for i, j in zip(ia.tolist(), ib.tolist())])
    # far pairs (up to 180 deg) hold the same absolute bound scaled by their size
    assert np.all(np.abs(got - wa) <= TOL * np.maximum(1.0, wa / 3600.0))
