"""Catalogues in different frames (Section 2: equatorial and galactic
coordinate systems).

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use this module (see the package
docstring); it shares no code with the GPU library.

Reading: when catalogue A's frame differs from catalogue B's, A's positions
(and the orientations of its areas) are first converted into B's frame by
a fixed FP64 rule (``c3o_frame_convert`` in c3x_oracle.c: correctly rounded
operations only, in a fixed order, so that any IEEE machine gets the same
bits), and the converted doubles are A's inputs of the cross-match in B's
frame. The rotation it applies is fixed by the galactic north pole at RA
192.85948 deg, Dec 27.12825 deg and the galactic longitude 122.93192 deg of
the north celestial pole, taken as exact decimals; its entries are the
nearest doubles to the exact values (here at 200 bits).
"""
from __future__ import annotations

import ctypes

import mpmath
import numpy as np

RA_GP, DEC_GP, L_NCP = "192.85948", "27.12825", "122.93192"
EQUATORIAL, GALACTIC = 0, 1


def _basis():
    """Galactic basis vectors x_G, y_G, z_G in equatorial coordinates, at
    200 bits: z_G the pole; the north celestial pole has galactic longitude
    L_NCP and latitude DEC_GP."""
    with mpmath.workprec(200):
        k = mpmath.pi / 180
        a, d, l = mpmath.mpf(RA_GP) * k, mpmath.mpf(DEC_GP) * k, mpmath.mpf(L_NCP) * k
        zg = [mpmath.cos(d) * mpmath.cos(a), mpmath.cos(d) * mpmath.sin(a), mpmath.sin(d)]
        ze = [mpmath.mpf(0), mpmath.mpf(0), mpmath.mpf(1)]
        q = [(ze[i] - mpmath.sin(d) * zg[i]) / mpmath.cos(d) for i in range(3)]
        qp = [zg[1] * q[2] - zg[2] * q[1], zg[2] * q[0] - zg[0] * q[2],
              zg[0] * q[1] - zg[1] * q[0]]
        xg = [mpmath.cos(l) * q[i] - mpmath.sin(l) * qp[i] for i in range(3)]
        yg = [mpmath.sin(l) * q[i] + mpmath.cos(l) * qp[i] for i in range(3)]
        return xg, yg, zg


def rotation(src: int, dst: int) -> np.ndarray:
    """The rule's 3 x 3 matrix (row-major doubles) taking unit vectors of
    frame src to frame dst: equatorial -> galactic has the galactic basis
    vectors as rows, galactic -> equatorial is its transpose; the identity
    for one frame."""
    if src == dst:
        return np.eye(3).reshape(-1)
    xg, yg, zg = _basis()
    M = [[float(v) for v in row] for row in (xg, yg, zg)]
    M = np.array(M)
    if src == GALACTIC:
        M = M.T
    return np.ascontiguousarray(M.reshape(-1))


def rotation_exact(src: int, dst: int):
    """The same rotation at 200 bits (mpmath matrix)."""
    xg, yg, zg = _basis()
    M = mpmath.matrix([xg, yg, zg])
    return M if src == EQUATORIAL else M.T


def convert(ra, dec, src: int, dst: int):
    """(ra', dec', gamma) of positions converted by the rule; gamma (degrees)
    turns an orientation measured in frame src into one in frame dst."""
    from . import _dp, lib
    ra = np.ascontiguousarray(ra, dtype=np.float64)
    dec = np.ascontiguousarray(dec, dtype=np.float64)
    n = ra.shape[0]
    ro, do, go = np.empty(n), np.empty(n), np.empty(n)
    M = rotation(src, dst)
    L = lib()
    L.c3o_frame_convert(_dp(M), _dp(ra), _dp(dec), n, _dp(ro), _dp(do), _dp(go))
    return ro, do, go


def match_mixed(raA, decA, frameA, raB, decB, frameB, shape=0, radius_arcsec=1.0, a=None,
                b=None, pa=None, pa_zero_deg=0.0, pa_sense=1, **kw):
    """The cross-match of A (frame frameA) against B (frame frameB): A
    converted into B's frame by the rule, each area's orientation
    T = pa_zero + pa_sense PA turned by the rule's gamma, then the
    single-frame match in B's frame."""
    from . import match
    if frameA == frameB:
        return match(raA, decA, raB, decB, shape=shape, radius_arcsec=radius_arcsec, a=a, b=b,
                     pa=pa, pa_zero_deg=pa_zero_deg, pa_sense=pa_sense, **kw)
    ra2, dec2, gam = convert(raA, decA, frameA, frameB)
    if shape in (1, 2):
        T = (pa_zero_deg + pa_sense * np.asarray(pa, dtype=np.float64)) + gam
        return match(ra2, dec2, raB, decB, shape=shape, a=a, b=b, pa=T, pa_zero_deg=0.0,
                     pa_sense=1, **kw)
    return match(ra2, dec2, raB, decB, shape=shape, radius_arcsec=radius_arcsec, **kw)
