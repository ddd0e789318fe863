"""Pins for the CPU oracle, against things other than itself.

* closed forms (tests/golden/closed_forms.tsv, exact rational answers);
* ellipses placed on a known bearing and distance with an independent
  200-bit destination formula;
* 200-bit brute force (oracle/exact.py decides every pair from the
  definition, no FP64 ladder) on small random and adversarial catalogues;
* invariants: brute force == zone partitioning for several zone heights,
  circle symmetry, ellipse(a = b) == circle, Dec and RA mirrors, radius
  monotonicity, best match in the set and minimal, rerun determinism.
"""
import math
import os

import numpy as np
import pytest

import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.tsv")


def load_closed_forms():
    rows = []
    with open(GOLD) as f:
        for line in f:
            if line.startswith("#"):
                continue
            p = line.rstrip("\n").split("\t")
            rows.append(dict(kind=p[0], raA=float(p[1]), decA=float(p[2]), raB=float(p[3]),
                             decB=float(p[4]), shape=int(p[5]), r=float(p[6]), a=float(p[7]),
                             b=float(p[8]), pa=float(p[9]), pz=float(p[10]), sense=int(p[11]),
                             inside=bool(int(p[12]))))
    return rows


CLOSED = load_closed_forms()


def test_closed_forms_fixture_is_balanced():
    kinds = {r["kind"] for r in CLOSED}
    assert {"meridian", "equator", "pole", "pole2", "ellipse_axis"} <= kinds
    for k in kinds:
        v = [r["inside"] for r in CLOSED if r["kind"] == k]
        assert any(v) and not all(v), k


def test_closed_forms_single_pair(oracle_lib):
    wrong = []
    n_amb = 0
    for r in CLOSED:
        k = oracle_lib.decide(r["raA"], r["decA"], r["raB"], r["decB"], r["shape"], r["r"], r["a"],
                              r["b"], r["pa"], r["pz"], r["sense"])
        n_amb += k == 2
        got = oracle_lib.decide_exact(r["raA"], r["decA"], r["raB"], r["decB"], r["shape"], r["r"],
                                      r["a"], r["b"], r["pa"], r["pz"], r["sense"])
        if got != r["inside"]:
            wrong.append(r)
    assert not wrong, wrong[:5]
    # the ulp-adjacent cases must actually reach the extended-precision path
    assert n_amb > len(CLOSED) // 4


@pytest.mark.parametrize("method", ["zones", "brute"])
def test_closed_forms_through_join(oracle_lib, method):
    """Each closed-form row as its own (A_k, B_k) pair inside one join: the
    diagonal pair (k, k) is present iff the closed form says inside."""
    groups = {}
    for idx, r in enumerate(CLOSED):
        key = (r["shape"], r["r"], r["pz"], r["sense"])
        groups.setdefault(key, []).append(r)
    for (shape, rad, pz, sense), rs in groups.items():
        raA = np.array([r["raA"] for r in rs])
        decA = np.array([r["decA"] for r in rs])
        raB = np.array([r["raB"] for r in rs])
        decB = np.array([r["decB"] for r in rs])
        kw = {}
        if shape == 1:
            kw = dict(a=np.array([r["a"] for r in rs]), b=np.array([r["b"] for r in rs]),
                      pa=np.array([r["pa"] for r in rs]), pa_zero_deg=pz, pa_sense=sense)
        res = oracle_lib.match(raA, decA, raB, decB, shape=shape, radius_arcsec=rad,
                               method=method, nthreads=3, **kw)
        diag = set(int(i) for i, j in zip(res.ia, res.ib) if i == j)
        want = set(k for k, r in enumerate(rs) if r["inside"])
        assert diag == want, (shape, rad, pz, sense)


def _dest_mp(ra, dec, bearing_deg, dist_deg):
    """Independent 200-bit destination formula (spherical trigonometry)."""
    import mpmath
    from mpmath import mpf
    with mpmath.workprec(200):
        k = mpmath.pi / 180
        d1 = mpf(dec) * k
        t = mpf(dist_deg) * k
        b = mpf(bearing_deg) * k
        sd2 = mpmath.sin(d1) * mpmath.cos(t) + mpmath.cos(d1) * mpmath.sin(t) * mpmath.cos(b)
        d2 = mpmath.asin(sd2)
        y = mpmath.sin(b) * mpmath.sin(t) * mpmath.cos(d1)
        x = mpmath.cos(t) - mpmath.sin(d1) * sd2
        ra2 = mpf(ra) + mpmath.atan2(y, x) / k
        ra2 = ra2 % 360
        return float(ra2), float(d2 / k)


@pytest.mark.parametrize("dec", [0.0, 33.3, -61.0, 80.0, 89.9])
def test_ellipse_known_pa(oracle_lib, dec):
    """B on the ellipse's own axes at distance (1 -+ 1e-9) times the axis, for
    orientations built from several zero-points and senses: inside then
    outside, whatever the latitude."""
    a, b = 20.0, 7.0
    cases = []
    for pz, sense, pa in ((0.0, 1, 30.0), (0.0, 1, 45.0), (90.0, -1, 30.0), (10.0, -1, -35.0),
                          (0.0, 1, 137.0)):
        T = pz + sense * pa
        for along, lim in ((0.0, a), (90.0, b), (180.0, a), (270.0, b)):
            for f, want in ((1 - 1e-9, True), (1 + 1e-9, False)):
                rb, db = _dest_mp(47.0, dec, T + along, lim / 3600.0 * f)
                cases.append((pz, sense, pa, rb, db, want))
    for pz, sense, pa, rb, db, want in cases:
        got = oracle_lib.decide_exact(47.0, dec, rb, db, 1, 0.0, a, b, pa, pz, sense)
        assert got == want, (dec, pz, sense, pa, rb, db)
        res = oracle_lib.match(np.array([47.0]), np.array([dec]), np.array([rb]), np.array([db]),
                               shape=1, a=np.array([a]), b=np.array([b]), pa=np.array([pa]),
                               pa_zero_deg=pz, pa_sense=sense)
        assert (len(res.ia) == 1) == want


def _near_boundary_catalogue(seed, nA, n_near, shape, radius=2.0, lat=(-89.0, 89.0)):
    g = np.random.default_rng(seed)
    raA, decA = synth.area_uniform(g, nA, 0.0, 360.0, *lat)
    par = g.integers(0, nA, n_near)
    if shape == 1:
        a = g.uniform(2.0, 30.0, nA)
        b = a * g.uniform(0.3, 1.0, nA)
        pa = g.uniform(0, 180, nA)
        reach = a[par]
    else:
        a = b = pa = None
        reach = np.full(n_near, radius)
    dist = reach * g.choice([0.3, 0.9, 0.999999, 1.0, 1.000001, 1.1, 2.0], n_near) / 3600.0
    rb, db = synth.destination(raA[par], decA[par], g.uniform(0, 360, n_near), dist)
    return raA, decA, rb, db, a, b, pa


@pytest.mark.parametrize("shape", [0, 1])
@pytest.mark.parametrize("lat", [(-89.0, 89.0), (88.0, 90.0), (-30.0, 30.0)])
def test_against_exact_brute_force(oracle_lib, shape, lat):
    raA, decA, raB, decB, a, b, pa = _near_boundary_catalogue(7 + shape, 40, 400, shape, lat=lat)
    kw = dict(a=a, b=b, pa=pa, pa_zero_deg=12.0, pa_sense=-1) if shape == 1 else {}
    pairs, best = oracle_lib.exact.brute(raA, decA, raB, decB, shape=shape, radius_arcsec=2.0, **kw)
    for method in ("zones", "brute"):
        res = oracle_lib.match(raA, decA, raB, decB, shape=shape, radius_arcsec=2.0, method=method,
                               nthreads=2, **kw)
        got = list(zip(res.ia.tolist(), res.ib.tolist()))
        assert got == sorted(pairs), method
        assert res.best_idx.tolist() == best, method
    assert len(pairs) > 60


def test_adversarial_against_exact(oracle_lib):
    c = synth.adversarial_circle(radius_arcsec=1.0, n_centres=24)
    pairs, best = oracle_lib.exact.brute(c.raA, c.decA, c.raB, c.decB, radius_arcsec=1.0)
    res = oracle_lib.match(c.raA, c.decA, c.raB, c.decB, radius_arcsec=1.0, nthreads=4)
    assert list(zip(res.ia.tolist(), res.ib.tolist())) == sorted(pairs)
    assert res.best_idx.tolist() == best
    assert res.n_ambiguous > 0      # the 2^-45 placements must reach the fallback


# ---------------------------------------------------------------------------- invariants

def _pairs(res):
    return set(zip(res.ia.tolist(), res.ib.tolist()))


@pytest.fixture(scope="module")
def small_cfg2():
    return synth.cfg2_fullsky(scale=0.0008)


def test_brute_equals_zones_several_heights(oracle_lib, small_cfg2):
    c = small_cfg2
    ref = oracle_lib.match(c.raA, c.decA, c.raB, c.decB, radius_arcsec=30.0, method="brute",
                           nthreads=8)
    assert len(ref.ia) > 1000
    for h in (30.0 / 3600, 90.0 / 3600, 10.0 / 3600, 1.0, 7.0):
        res = oracle_lib.match(c.raA, c.decA, c.raB, c.decB, radius_arcsec=30.0, method="zones",
                               zone_deg=h, nthreads=5)
        assert np.array_equal(res.ia, ref.ia) and np.array_equal(res.ib, ref.ib), h
        assert np.array_equal(res.best_idx, ref.best_idx)
        assert np.array_equal(res.sep, ref.sep)


def test_circle_symmetry(oracle_lib, small_cfg2):
    c = small_cfg2
    ab = oracle_lib.match(c.raA, c.decA, c.raB, c.decB, radius_arcsec=30.0)
    ba = oracle_lib.match(c.raB, c.decB, c.raA, c.decA, radius_arcsec=30.0)
    assert _pairs(ab) == {(j, i) for i, j in _pairs(ba)}


def test_ellipse_with_equal_axes_is_circle(oracle_lib, small_cfg2):
    c = small_cfg2
    n = c.nA
    circ = oracle_lib.match(c.raA, c.decA, c.raB, c.decB, radius_arcsec=30.0)
    g = np.random.default_rng(3)
    ell = oracle_lib.match(c.raA, c.decA, c.raB, c.decB, shape=1, a=np.full(n, 30.0),
                           b=np.full(n, 30.0), pa=g.uniform(-360, 360, n), pa_zero_deg=17.0,
                           pa_sense=-1)
    assert _pairs(circ) == _pairs(ell)


def test_mirrors(oracle_lib):
    c = synth.cfg3_galactic_ellipses(scale=0.0004)
    kw = dict(shape=1, a=c.a_arcsec, b=c.b_arcsec, pa=c.pa_deg)
    # keep RA in [180, 360) so that 360 - RA is exact
    raA = 180.0 + c.raA * 0.5
    raB = 180.0 + c.raB * 0.5
    base = oracle_lib.match(raA, c.decA, raB, c.decB, pa_zero_deg=20.0, pa_sense=1, **kw)
    assert len(base.ia) > 100
    dm = oracle_lib.match(raA, -c.decA, raB, -c.decB, pa_zero_deg=160.0, pa_sense=-1, **kw)
    assert _pairs(base) == _pairs(dm)
    rm = oracle_lib.match(360.0 - raA, c.decA, 360.0 - raB, c.decB, pa_zero_deg=-20.0,
                          pa_sense=-1, **kw)
    assert _pairs(base) == _pairs(rm)


def test_radius_monotone_and_best_minimal(oracle_lib, small_cfg2):
    c = small_cfg2
    prev = set()
    for r in (1.0, 5.0, 30.0, 120.0):
        res = oracle_lib.match(c.raA, c.decA, c.raB, c.decB, radius_arcsec=r)
        cur = _pairs(res)
        assert prev <= cur
        prev = cur
        for i in np.unique(res.ia)[:500].tolist():
            sel = res.ia == i
            j = res.best_idx[i]
            assert j in set(res.ib[sel].tolist())
            assert res.best_sep[i] == res.sep[sel].min()
        unmatched = np.setdiff1d(np.arange(c.nA), res.ia)
        assert np.all(res.best_idx[unmatched] == -1)


def test_rerun_is_byte_identical(oracle_lib, small_cfg2):
    c = small_cfg2
    r1 = oracle_lib.match(c.raA, c.decA, c.raB, c.decB, radius_arcsec=60.0, nthreads=7)
    r2 = oracle_lib.match(c.raA, c.decA, c.raB, c.decB, radius_arcsec=60.0, nthreads=2)
    for f in ("ia", "ib", "sep", "best_idx"):
        assert getattr(r1, f).tobytes() == getattr(r2, f).tobytes()


def test_duplicates_and_zero_radius(oracle_lib):
    raA = np.array([10.0, 0.0, 0.0, 359.5])
    decA = np.array([20.0, 90.0, -90.0, 0.0])
    raB = np.array([10.0, 10.0, 123.0, 0.0, 359.5, 359.5])
    decB = np.array([20.0, 20.0, 90.0, -90.0, 0.0, 1e-300])
    res = oracle_lib.match(raA, decA, raB, decB, radius_arcsec=0.0)
    # same point: equal coordinates, or both on the same pole at any RA
    assert _pairs(res) == {(0, 0), (0, 1), (1, 2), (2, 3), (3, 4)}
    assert res.best_idx.tolist() == [0, 2, 3, 4]      # exact tie -> lower index
    res = oracle_lib.match(raA, decA, raB, decB, radius_arcsec=1.0)
    assert (3, 5) in _pairs(res)


def test_validation(oracle_lib):
    ok = np.array([1.0])
    with pytest.raises(ValueError):
        oracle_lib.match(np.array([360.0]), ok, ok, ok)
    with pytest.raises(ValueError):
        oracle_lib.match(ok, np.array([90.5]), ok, ok)
    with pytest.raises(ValueError):
        oracle_lib.match(ok, ok, np.array([np.nan]), ok)
    with pytest.raises(ValueError):
        oracle_lib.match(ok, ok, ok, ok, radius_arcsec=-1.0)
    with pytest.raises(ValueError):
        oracle_lib.match(ok, ok, ok, ok, shape=1, a=ok, b=np.array([2.0]), pa=ok)
    with pytest.raises(ValueError):
        oracle_lib.match(ok, ok, ok, ok, pa_sense=0)


def test_cfg1_pair_count_sanity(oracle_lib):
    """~7,000 jittered copies (sigma 0.3" << r = 1") plus ~26 chance pairs."""
    c = synth.cfg1_patch()
    res = oracle_lib.match(c.raA, c.decA, c.raB, c.decB, radius_arcsec=1.0)
    assert 6950 <= len(res.ia) <= 7060
    # brute force over the whole 10k x 10k (1e8 tests) agrees
    bf = oracle_lib.match(c.raA, c.decA, c.raB, c.decB, radius_arcsec=1.0, method="brute",
                          nthreads=8)
    assert _pairs(bf) == _pairs(res)
    assert np.array_equal(bf.best_idx, res.best_idx)
