"""Pins of the oracle's concentric ellipses (Section 3, ClumpPopulator): B
sources placed exactly on an ellipse axis (levels known in closed form), a
200-bit brute force on tiny random inputs, and the nesting of the scales."""
import json
import os

import numpy as np
import pytest

from oracle import concentric as C

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "concentric_axes.json")


def axis_catalogue(ex, case):
    """A on the equator at the listed RAs; B at distance d along the case's
    direction from each A."""
    raA = np.array(ex["ra_centres"], dtype=np.float64)
    decA = np.zeros_like(raA)
    raB, decB, want = [], [], []
    for i, r0 in enumerate(ex["ra_centres"]):
        for d, lv in zip(case["d_arcsec"], case["level"]):
            dd = d / 3600.0
            ra, de = {"north": (r0, dd), "south": (r0, -dd), "east": (r0 + dd, 0.0),
                      "west": (r0 - dd, 0.0)}[case["dir"]]
            if lv is not None:
                want.append((i, len(raB), lv))
            raB.append(ra)
            decB.append(de)
    return raA, decA, np.array(raB), np.array(decB), want


@pytest.mark.parametrize("ci", range(6))
def test_levels_on_the_axes(ci):
    ex = json.load(open(GOLDEN))
    case = ex["cases"][ci]
    raA, decA, raB, decB, want = axis_catalogue(ex, case)
    n = raA.size
    a = np.full(n, ex["a_arcsec"])
    b = np.full(n, ex["b_arcsec"])
    pa = np.full(n, case["pa_deg"])
    c = C.concentric(raA, decA, raB, decB, a, b, pa, ex["scales"])
    got = list(zip(c.ia.tolist(), c.ib.tolist(), c.level.tolist()))
    assert got == want


def test_brute_force_tiny():
    rng = np.random.default_rng(3)
    scales = [0.4, 0.8, 1.0, 1.7]
    for trial in range(4):
        nA, nB = 4, 40
        ra0 = rng.uniform(0, 360)
        de0 = rng.uniform(-80, 80)
        raA = (ra0 + rng.uniform(-0.01, 0.01, nA)) % 360.0
        decA = de0 + rng.uniform(-0.01, 0.01, nA)
        raB = (ra0 + rng.uniform(-0.012, 0.012, nB)) % 360.0
        decB = de0 + rng.uniform(-0.012, 0.012, nB)
        a = rng.uniform(5.0, 25.0, nA)
        b = a * rng.uniform(0.3, 1.0, nA)
        pa = rng.uniform(0, 180, nA)
        c = C.concentric(raA, decA, raB, decB, a, b, pa, scales, pa_zero_deg=90.0, pa_sense=-1)
        got = list(zip(c.ia.tolist(), c.ib.tolist(), c.level.tolist()))
        want = C.levels_brute(raA, decA, raB, decB, a, b, pa, scales, 90.0, -1)
        assert got == want
        assert len(want) > 0


def test_nesting_and_single_scale():
    """Level <= m is exactly the pair set of scale m's own match; one scale
    of 1 is the plain elliptical match."""
    import oracle
    import synth
    cat = synth.cfg3_galactic_ellipses(scale=0.0005)
    kw = dict(pa_zero_deg=cat.pa_zero_deg, pa_sense=cat.pa_sense)
    scales = [0.5, 1.0, 2.0]
    c = C.concentric(cat.raA, cat.decA, cat.raB, cat.decB, cat.a_arcsec, cat.b_arcsec,
                     cat.pa_deg, scales, **kw)
    for m, k in enumerate(scales):
        o = oracle.match(cat.raA, cat.decA, cat.raB, cat.decB, shape=1, a=cat.a_arcsec * k,
                         b=cat.b_arcsec * k, pa=cat.pa_deg, **kw)
        sel = c.level <= m
        assert np.array_equal(c.ia[sel], o.ia) and np.array_equal(c.ib[sel], o.ib)
    one = C.concentric(cat.raA, cat.decA, cat.raB, cat.decB, cat.a_arcsec, cat.b_arcsec,
                       cat.pa_deg, [1.0], **kw)
    assert np.all(one.level == 0) and len(one.ia) > 0
    assert len(np.unique(c.level)) == 3
    with pytest.raises(ValueError):
        C.check_scales([1.0, 1.0])
    with pytest.raises(ValueError):
        C.check_scales([0.0, 1.0])
