"""CPU oracle for the positional cross-match.

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. The GPU library
(``paper_1611_08494_amd``) never imports it, and the two share no code.

``match`` follows the paper's "Sky" functional case (Section 2.1) with the
"all" and "best" match selections (Section 2.2): the plain C library
(``c3x_oracle.c``) decides every candidate in FP64 with a proven error bound,
returns the pairs it could not certify as ambiguous, and ``exact.py`` decides
those at 200 bits. Best matches are the exact argmin of (theta, j) over each
row's matches; FP64 separations closer than 2^-38 (relative) are re-ranked at
200 bits.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import Optional

import numpy as np

from . import exact

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "c3x_oracle.c")
_LIB = os.path.join(_HERE, "_build", "libc3x_oracle.so")


def build(force: bool = True) -> str:
    """Compile the C oracle (gcc -O2, no fast-math)."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared",
                        "-Wall", "-o", tmp, _SRC, "-lm", "-lpthread"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Out(ctypes.Structure):
    _fields_ = [
        ("n_in", ctypes.c_int64),
        ("in_a", ctypes.POINTER(ctypes.c_int32)),
        ("in_b", ctypes.POINTER(ctypes.c_int32)),
        ("in_sep", ctypes.POINTER(ctypes.c_double)),
        ("n_amb", ctypes.c_int64),
        ("amb_a", ctypes.POINTER(ctypes.c_int32)),
        ("amb_b", ctypes.POINTER(ctypes.c_int32)),
        ("n_tests", ctypes.c_int64),
        ("threads_used", ctypes.c_int32),
    ]


class _Area(ctypes.Structure):
    _fields_ = [
        ("shape", ctypes.c_int),
        ("radius_arcsec", ctypes.c_double),
        ("a_arcsec", ctypes.POINTER(ctypes.c_double)),
        ("b_arcsec", ctypes.POINTER(ctypes.c_double)),
        ("pa_deg", ctypes.POINTER(ctypes.c_double)),
        ("pa_zero_deg", ctypes.c_double),
        ("pa_sense", ctypes.c_int),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.c3o_match.argtypes = [dp, dp, ctypes.c_int64, dp, dp, ctypes.c_int64,
                                ctypes.POINTER(_Area), ctypes.c_int, ctypes.c_double,
                                ctypes.c_int, ctypes.POINTER(_Out)]
        L.c3o_match.restype = ctypes.c_int
        L.c3o_free.argtypes = [ctypes.POINTER(_Out)]
        L.c3o_decide.argtypes = [ctypes.c_double] * 4 + [ctypes.POINTER(_Area), ctypes.c_int64]
        L.c3o_decide.restype = ctypes.c_int
        ip = ctypes.POINTER(ctypes.c_int32)
        L.c3o_seps.argtypes = [dp, dp, dp, dp, ip, ip, ctypes.c_int64, dp]
        L.c3o_frame_convert.argtypes = [dp, dp, dp, ctypes.c_int64, dp, dp, dp]
        L.c3o_frame_convert.restype = None
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclasses.dataclass
class Result:
    ia: np.ndarray          # int32, canonical (ia, ib) order
    ib: np.ndarray          # int32
    sep: np.ndarray         # float64 arcsec
    best_idx: np.ndarray    # int32 per A row, -1 if unmatched
    best_sep: np.ndarray    # float64 per A row, NaN if unmatched
    n_ambiguous: int
    n_best_ties: int
    n_tests: int
    threads: int


def _area(shape, radius_arcsec, a, b, pa, pa_zero_deg, pa_sense):
    ar = _Area()
    ar.shape = int(shape)
    ar.radius_arcsec = float(radius_arcsec)
    ar.pa_zero_deg = float(pa_zero_deg)
    ar.pa_sense = int(pa_sense)
    keep = []
    if shape in (1, 2):
        for name, v in (("a_arcsec", a), ("b_arcsec", b), ("pa_deg", pa)):
            v = np.ascontiguousarray(v, dtype=np.float64)
            keep.append(v)
            setattr(ar, name, _dp(v))
    return ar, keep


def validate(raA, decA, raB, decB, shape, radius_arcsec, a, b, pa, pa_sense):
    """Input domain of the cross-match: RA in [0, 360), |Dec| <= 90, finite;
    radius 0 or in [1e-6", 90 deg]; ellipse semi-axes or rectangle half-sides
    1e-6" <= b <= a <= 90 deg, a/b <= 1000, PA finite; pa_sense +1 or -1."""
    for name, ra, de in (("A", raA, decA), ("B", raB, decB)):
        if not (np.all(np.isfinite(ra)) and np.all(np.isfinite(de))):
            raise ValueError(f"catalogue {name}: non-finite coordinate")
        if ra.size and (ra.min() < 0.0 or ra.max() >= 360.0):
            raise ValueError(f"catalogue {name}: RA outside [0, 360)")
        if de.size and (np.abs(de).max() > 90.0):
            raise ValueError(f"catalogue {name}: |Dec| > 90")
    if pa_sense not in (1, -1):
        raise ValueError("pa_sense must be +1 or -1")
    if shape not in (0, 1, 2):
        raise ValueError("shape must be 0 (circle), 1 (ellipse) or 2 (rectangle)")
    if shape == 0:
        r = float(radius_arcsec)
        if not (r == 0.0 or (1e-6 <= r <= 324000.0)):
            raise ValueError("radius must be 0 or in [1e-6, 324000] arcsec")
    else:
        a = np.asarray(a, dtype=np.float64)
        b = np.asarray(b, dtype=np.float64)
        pa = np.asarray(pa, dtype=np.float64)
        if a.shape != raA.shape or b.shape != raA.shape or pa.shape != raA.shape:
            raise ValueError("ellipse parameters must have one entry per A row")
        if a.size:
            if not (np.all(np.isfinite(a)) and np.all(np.isfinite(b)) and np.all(np.isfinite(pa))):
                raise ValueError("non-finite ellipse parameter")
            if b.min() < 1e-6 or np.any(b > a) or a.max() > 324000.0 or np.any(a > 1000.0 * b):
                raise ValueError("ellipse axes outside 1e-6 <= b <= a <= 324000, a/b <= 1000")


def match(raA, decA, raB, decB, shape: int = 0, radius_arcsec: float = 1.0,
          a=None, b=None, pa=None, pa_zero_deg: float = 0.0, pa_sense: int = 1,
          method: str = "zones", zone_deg: Optional[float] = None,
          nthreads: Optional[int] = None) -> Result:
    """All matches plus the best match per A row (exact semantics)."""
    raA = np.ascontiguousarray(raA, dtype=np.float64)
    decA = np.ascontiguousarray(decA, dtype=np.float64)
    raB = np.ascontiguousarray(raB, dtype=np.float64)
    decB = np.ascontiguousarray(decB, dtype=np.float64)
    validate(raA, decA, raB, decB, shape, radius_arcsec, a, b, pa, pa_sense)
    nA, nB = raA.shape[0], raB.shape[0]
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    if zone_deg is None:
        if shape == 2 and nA:
            reach = float(np.max(np.hypot(a, b))) / 3600.0
        else:
            reach = (float(np.max(a)) if (shape == 1 and nA) else float(radius_arcsec)) / 3600.0
        zone_deg = max(reach, 180.0 / 4_000_000)
    ar, keep = _area(shape, radius_arcsec, a, b, pa, pa_zero_deg, pa_sense)
    out = _Out()
    rc = lib().c3o_match(_dp(raA), _dp(decA), nA, _dp(raB), _dp(decB), nB, ctypes.byref(ar),
                         0 if method == "brute" else 1, float(zone_deg), int(nthreads),
                         ctypes.byref(out))
    if rc != 0:
        raise RuntimeError(f"oracle c3o_match failed ({rc})")
    try:
        n_in, n_amb = out.n_in, out.n_amb
        ia = np.ctypeslib.as_array(out.in_a, (max(n_in, 1),))[:n_in].copy()
        ib = np.ctypeslib.as_array(out.in_b, (max(n_in, 1),))[:n_in].copy()
        sep = np.ctypeslib.as_array(out.in_sep, (max(n_in, 1),))[:n_in].copy()
        aa = np.ctypeslib.as_array(out.amb_a, (max(n_amb, 1),))[:n_amb].copy()
        ab = np.ctypeslib.as_array(out.amb_b, (max(n_amb, 1),))[:n_amb].copy()
        n_tests, threads = int(out.n_tests), int(out.threads_used)
    finally:
        lib().c3o_free(ctypes.byref(out))
    # re-decide the pairs FP64 could not certify
    keep_amb = []
    for i, j in zip(aa.tolist(), ab.tolist()):
        if shape == 1:
            ok = exact.decide_ellipse(raA[i], decA[i], raB[j], decB[j], a[i], b[i], pa[i],
                                      pa_zero_deg, pa_sense)
        elif shape == 2:
            ok = exact.decide_rect(raA[i], decA[i], raB[j], decB[j], a[i], b[i], pa[i],
                                   pa_zero_deg, pa_sense)
        else:
            ok = exact.decide_circle(raA[i], decA[i], raB[j], decB[j], radius_arcsec)
        keep_amb.append(ok)
    keep_amb = np.asarray(keep_amb, dtype=bool)
    if keep_amb.any():
        xa = aa[keep_amb].astype(np.int32)
        xb = ab[keep_amb].astype(np.int32)
        xs = np.empty(xa.shape[0], dtype=np.float64)
        ip = ctypes.POINTER(ctypes.c_int32)
        lib().c3o_seps(_dp(raA), _dp(decA), _dp(raB), _dp(decB), xa.ctypes.data_as(ip),
                       xb.ctypes.data_as(ip), xa.shape[0], _dp(xs))
        ia = np.concatenate([ia, xa])
        ib = np.concatenate([ib, xb])
        sep = np.concatenate([sep, xs])
    order = np.lexsort((ib, ia))
    ia, ib, sep = ia[order].astype(np.int32), ib[order].astype(np.int32), sep[order]
    best_idx, best_sep, n_ties = _best(raA, decA, raB, decB, ia, ib, sep, nA)
    return Result(ia, ib, sep, best_idx, best_sep, int(n_amb), n_ties, n_tests, threads)


def _best(raA, decA, raB, decB, ia, ib, sep, nA):
    best_idx = np.full(nA, -1, dtype=np.int32)
    best_sep = np.full(nA, np.nan)
    if ia.size == 0:
        return best_idx, best_sep, 0
    # per-row minimum separation, then (sep, ib) lexicographic minimum
    order = np.lexsort((ib, sep, ia))
    sa, sb, ss = ia[order], ib[order], sep[order]
    first = np.ones(sa.shape[0], dtype=bool)
    first[1:] = sa[1:] != sa[:-1]
    rows = sa[first]
    best_idx[rows] = sb[first]
    best_sep[rows] = ss[first]
    # near-ties: another match of the same row within 2^-38 (relative)
    mins = np.empty(nA)
    mins[rows] = ss[first]
    near = ss <= mins[sa] * (1.0 + 2.0 ** -38) + 1e-300
    near &= ~first
    tie_rows = np.unique(sa[near])
    for i in tie_rows.tolist():
        m = mins[i]
        sel = (ia == i) & (sep <= m * (1.0 + 2.0 ** -38) + 1e-300)
        cand = [(int(j), raB[j], decB[j]) for j in ib[sel].tolist()]
        j = exact.best_of(raA[i], decA[i], cand)
        best_idx[i] = j
        best_sep[i] = sep[(ia == i) & (ib == j)][0]
    return best_idx, best_sep, int(tie_rows.shape[0])


def seps(raA, decA, raB, decB, ia, ib) -> np.ndarray:
    """The oracle's FP64 separation (arcsec) of the pairs (ia[k], ib[k])."""
    raA, decA, raB, decB = (np.ascontiguousarray(v, dtype=np.float64)
                            for v in (raA, decA, raB, decB))
    ia = np.ascontiguousarray(ia, dtype=np.int32)
    ib = np.ascontiguousarray(ib, dtype=np.int32)
    out = np.empty(ia.shape[0], dtype=np.float64)
    ip = ctypes.POINTER(ctypes.c_int32)
    lib().c3o_seps(_dp(raA), _dp(decA), _dp(raB), _dp(decB), ia.ctypes.data_as(ip),
                   ib.ctypes.data_as(ip), ia.shape[0], _dp(out))
    return out


def decide(ra1, dec1, ra2, dec2, shape=0, radius_arcsec=1.0, a=0.0, b=0.0, pa=0.0,
           pa_zero_deg=0.0, pa_sense=1) -> int:
    """FP64 certified decision of one pair: 0 out, 1 in, 2 ambiguous."""
    av = np.array([a], dtype=np.float64)
    bv = np.array([b], dtype=np.float64)
    pv = np.array([pa], dtype=np.float64)
    ar, keep = _area(shape, radius_arcsec, av, bv, pv, pa_zero_deg, pa_sense)
    return int(lib().c3o_decide(float(ra1), float(dec1), float(ra2), float(dec2),
                                ctypes.byref(ar), 0))


def decide_exact(ra1, dec1, ra2, dec2, shape=0, radius_arcsec=1.0, a=0.0, b=0.0, pa=0.0,
                 pa_zero_deg=0.0, pa_sense=1) -> bool:
    """Certified decision, falling back to 200-bit arithmetic when FP64 cannot
    certify it."""
    k = decide(ra1, dec1, ra2, dec2, shape, radius_arcsec, a, b, pa, pa_zero_deg, pa_sense)
    if k != 2:
        return k == 1
    if shape == 1:
        return exact.decide_ellipse(ra1, dec1, ra2, dec2, a, b, pa, pa_zero_deg, pa_sense)
    if shape == 2:
        return exact.decide_rect(ra1, dec1, ra2, dec2, a, b, pa, pa_zero_deg, pa_sense)
    return exact.decide_circle(ra1, dec1, ra2, dec2, radius_arcsec)
