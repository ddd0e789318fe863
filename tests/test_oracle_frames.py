"""Pins for the oracle's frame conversion (oracle/frames.py; paper Section
2: catalogues in equatorial or galactic coordinates), the reading under
which a catalogue in another frame is first converted by a fixed FP64 rule:

* the rule against the exact rotation (200-bit mpmath, independent of the
  rule's own arithmetic): positions within 1e-11 deg everywhere, the poles
  and the RA seam included;
* points fixed by the frame definition: the north celestial pole lands at
  galactic (122.93192, 27.12825), the galactic north pole at b = 90, the
  galactic centre near (266.405, -28.936);
* round trips equatorial -> galactic -> equatorial within 1e-11 deg;
* the orientation turn gamma equals the bearing (at 200 bits) of a point
  due north of the source in the source frame, seen in the target frame;
* mixed-frame matches decide every pair further than 1e-8 arcsec from the
  boundary as the exact rotation does.
"""
import mpmath
import numpy as np
import pytest

import synth
from oracle import exact, frames

EQ, GAL = frames.EQUATORIAL, frames.GALACTIC


def _exact_convert(ra, dec, src, dst):
    M = frames.rotation_exact(src, dst)
    with mpmath.workprec(200):
        k = mpmath.pi / 180
        a, d = mpmath.mpf(float(ra)) * k, mpmath.mpf(float(dec)) * k
        p = mpmath.matrix([mpmath.cos(d) * mpmath.cos(a), mpmath.cos(d) * mpmath.sin(a),
                           mpmath.sin(d)])
        q = M * p
        ra2 = mpmath.atan2(q[1], q[0]) / k % 360
        dec2 = mpmath.atan2(q[2], mpmath.sqrt(q[0] ** 2 + q[1] ** 2)) / k
        return ra2, dec2


def _angle_deg(ra1, dec1, ra2, dec2):
    return float(exact.theta(float(ra1), float(dec1), float(ra2), float(dec2)) * 180 / mpmath.pi)


@pytest.mark.parametrize("src,dst", [(EQ, GAL), (GAL, EQ)])
def test_rule_against_exact_rotation(src, dst):
    g = np.random.default_rng(1)
    ra, dec = synth.sphere_uniform(g, 300)
    ra = np.concatenate([ra, [0.0, 359.9999999, 123.0, 45.0, 0.0, 266.4]])
    dec = np.concatenate([dec, [90.0, -90.0, 89.9999999, -89.99999, 0.0, -28.9]])
    r2, d2, _ = frames.convert(ra, dec, src, dst)
    assert np.all((r2 >= 0.0) & (r2 < 360.0)) and np.all(np.abs(d2) <= 90.0)
    worst = 0.0
    for k in range(len(ra)):
        er, ed = _exact_convert(ra[k], dec[k], src, dst)
        worst = max(worst, _angle_deg(r2[k], d2[k], float(er), float(ed)))
    assert worst < 1e-11, worst


def test_defining_points():
    r, d, _ = frames.convert(np.array([0.0, 77.0]), np.array([90.0, 90.0]), EQ, GAL)
    assert np.allclose(r, 122.93192, atol=1e-11) and np.allclose(d, 27.12825, atol=1e-11)
    r, d, _ = frames.convert(np.array([192.85948]), np.array([27.12825]), EQ, GAL)
    assert abs(d[0] - 90.0) < 1e-11
    r, d, _ = frames.convert(np.array([0.0]), np.array([0.0]), GAL, EQ)
    assert abs(r[0] - 266.405) < 1e-3 and abs(d[0] + 28.936) < 1e-3


def test_round_trip():
    g = np.random.default_rng(2)
    ra, dec = synth.sphere_uniform(g, 2000)
    r2, d2, _ = frames.convert(ra, dec, EQ, GAL)
    r3, d3, _ = frames.convert(r2, d2, GAL, EQ)
    for k in range(0, 2000, 97):
        assert _angle_deg(ra[k], dec[k], r3[k], d3[k]) < 1e-11


@pytest.mark.parametrize("src,dst", [(EQ, GAL), (GAL, EQ)])
def test_orientation_turn(src, dst):
    """gamma: the source frame's north at the point, as a bearing (from the
    target frame's north towards its east) in the target frame."""
    g = np.random.default_rng(3)
    ra, dec = synth.sphere_uniform(g, 40)
    dec = np.clip(dec, -80, 80)
    r2, d2, gam = frames.convert(ra, dec, src, dst)
    M = frames.rotation_exact(src, dst)
    for k in range(len(ra)):
        with mpmath.workprec(200):
            kk = mpmath.pi / 180
            a, d = mpmath.mpf(float(ra[k])) * kk, mpmath.mpf(float(dec[k])) * kk
            north = mpmath.matrix([-mpmath.sin(d) * mpmath.cos(a), -mpmath.sin(d) * mpmath.sin(a),
                                   mpmath.cos(d)])
            nq = M * north
            a2, d2e = _exact_convert(ra[k], dec[k], src, dst)
            a2, d2e = a2 * kk, d2e * kk
            east = mpmath.matrix([-mpmath.sin(a2), mpmath.cos(a2), 0])
            nth = mpmath.matrix([-mpmath.sin(d2e) * mpmath.cos(a2), -mpmath.sin(d2e) *
                                 mpmath.sin(a2), mpmath.cos(d2e)])
            want = float(mpmath.atan2(sum(nq[i] * east[i] for i in range(3)),
                                      sum(nq[i] * nth[i] for i in range(3))) / kk)
        diff = (gam[k] - want + 180.0) % 360.0 - 180.0
        assert abs(diff) < 1e-9, (k, gam[k], want)


def test_mixed_frame_match_against_exact_rotation(oracle_lib):
    g = np.random.default_rng(4)
    raA, decA = synth.cap_uniform(g, 400, 150.0, 40.0, 0.02)
    raB, decB = synth.cap_uniform(g, 600, 150.0, 40.0, 0.02)
    rB2, dB2, _ = frames.convert(raB, decB, EQ, GAL)   # B given in the galactic frame
    r = 10.0
    res = frames.match_mixed(raA, decA, EQ, rB2, dB2, GAL, radius_arcsec=r)
    got = set(zip(res.ia.tolist(), res.ib.tolist()))
    assert len(got) > 200
    # exact rotation of A into the galactic frame, exact angles to B
    M = frames.rotation_exact(EQ, GAL)
    checked = 0
    for i in range(0, len(raA), 7):
        ea, ed = _exact_convert(raA[i], decA[i], EQ, GAL)
        for j in range(len(raB)):
            with mpmath.workprec(200):
                k = mpmath.pi / 180
                th = exact.theta(float(ea), float(ed), rB2[j], dB2[j])  # near-exact point
            t = float(th * 180 / mpmath.pi * 3600)
            if abs(t - r) > 1e-8:
                assert ((i, j) in got) == (t < r), (i, j, t)
                checked += 1
    assert checked > 10000
