"""Seeded synthetic catalogues standing in for the survey data the paper uses.

The paper validates its tool on real public catalogues and uses Hi-GAL clumps
against UKIDSS/GLIMPSE sources (ViaLactea, Section 3); none of those data are
available here. These generators draw catalogues with the shapes, sizes and
density structure of the workloads the cross-match is measured on:

* ``cfg1_patch``      10k x 10k on a 1 deg x 1 deg equatorial patch, r = 1".
* ``cfg2_fullsky``    10M x 10M full sky plus two dense 1M caps (one straddling
                      RA = 0/360, one containing the north pole), r = 2".
* ``cfg3_galactic_ellipses``  100k clumps with per-source ellipses against 50M
                      point sources in the galactic band, galactic frame.
* ``cfg4_jobs``       4096 independent small cross-matches (batched form).
* ``cfg5_scale``      200M x 200M full sky with galactic-plane clustering.

Every config takes a ``scale`` factor that shrinks all counts (areas and
densities of the dense parts are kept where that makes sense), so the CPU test
suite can run the same recipes at small sizes.

Conventions: angles in degrees (float64), RA in [0, 360), Dec in [-90, 90].
"Area-uniform" in a RA/Dec box means RA ~ U[lo, hi) and Dec = asin(U[sin lo,
sin hi)). A cap of radius rho is sampled as theta = acos(U[cos rho, 1]) with a
uniform bearing about its centre. "Jitter sigma" is an isotropic tangent-plane
Gaussian with sigma per axis, applied with the great-circle destination formula.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

SEED_BASE = 1611084940
D2R = math.pi / 180.0
ARCSEC = 1.0 / 3600.0


@dataclasses.dataclass
class Catalogues:
    """One cross-match workload: catalogue A (centres), catalogue B, area."""

    name: str
    raA: np.ndarray
    decA: np.ndarray
    raB: np.ndarray
    decB: np.ndarray
    frame: int = 0                 # 0 equatorial, 1 galactic
    shape: int = 0                 # 0 circle, 1 ellipse, 2 rectangle
    radius_arcsec: float = 1.0
    a_arcsec: Optional[np.ndarray] = None
    b_arcsec: Optional[np.ndarray] = None
    pa_deg: Optional[np.ndarray] = None
    pa_zero_deg: float = 0.0
    pa_sense: int = 1
    # batched form: rows of (a_off, nA, b_off, nB, radius_arcsec)
    jobs: Optional[np.ndarray] = None
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def nA(self) -> int:
        return int(self.raA.shape[0])

    @property
    def nB(self) -> int:
        return int(self.raB.shape[0])

    def reach_arcsec(self) -> float:
        if self.shape == 1:
            return float(self.a_arcsec.max()) if self.nA else 0.0
        if self.shape == 2:  # rectangle: the half-diagonal
            return float(np.hypot(self.a_arcsec, self.b_arcsec).max()) if self.nA else 0.0
        if self.jobs is not None and len(self.jobs):
            return float(self.jobs[:, 4].max())
        return float(self.radius_arcsec)


# ----------------------------------------------------------------------------
# primitive samplers
# ----------------------------------------------------------------------------

def _norm_ra(ra: np.ndarray) -> np.ndarray:
    ra = np.mod(ra, 360.0)
    ra[ra >= 360.0] = 0.0           # mod can round up to exactly 360
    return ra


def area_uniform(rng: np.random.Generator, n: int, ra_lo: float, ra_hi: float,
                 dec_lo: float, dec_hi: float):
    """n points uniform in solid angle over a RA/Dec box (degrees)."""
    ra = rng.uniform(ra_lo, ra_hi, n)
    s = rng.uniform(math.sin(dec_lo * D2R), math.sin(dec_hi * D2R), n)
    dec = np.degrees(np.arcsin(np.clip(s, -1.0, 1.0)))
    return _norm_ra(ra), np.clip(dec, -90.0, 90.0)


def destination(ra: np.ndarray, dec: np.ndarray, bearing_deg: np.ndarray,
                dist_deg: np.ndarray):
    """Point reached from (ra, dec) after dist along a great circle leaving at
    the given bearing (from north towards east). Degrees in and out."""
    d1 = dec * D2R
    t = dist_deg * D2R
    b = bearing_deg * D2R
    sd2 = np.sin(d1) * np.cos(t) + np.cos(d1) * np.sin(t) * np.cos(b)
    d2 = np.arcsin(np.clip(sd2, -1.0, 1.0))
    y = np.sin(b) * np.sin(t) * np.cos(d1)
    x = np.cos(t) - np.sin(d1) * sd2
    ra2 = ra + np.degrees(np.arctan2(y, x))
    return _norm_ra(ra2), np.clip(np.degrees(d2), -90.0, 90.0)


def cap_uniform(rng: np.random.Generator, n: int, ra_c: float, dec_c: float,
                rho_deg: float):
    """n points uniform in solid angle inside a cap of radius rho."""
    u = rng.uniform(math.cos(rho_deg * D2R), 1.0, n)
    theta = np.degrees(np.arccos(np.clip(u, -1.0, 1.0)))
    bearing = rng.uniform(0.0, 360.0, n)
    return destination(np.full(n, ra_c), np.full(n, dec_c), bearing, theta)


def sphere_uniform(rng: np.random.Generator, n: int):
    return area_uniform(rng, n, 0.0, 360.0, -90.0, 90.0)


def jitter(rng: np.random.Generator, ra: np.ndarray, dec: np.ndarray,
           sigma_arcsec: float):
    """Isotropic tangent-plane Gaussian offset, sigma per axis."""
    n = ra.shape[0]
    dn = rng.normal(0.0, sigma_arcsec, n)
    de = rng.normal(0.0, sigma_arcsec, n)
    dist = np.hypot(dn, de) * ARCSEC
    bearing = np.degrees(np.arctan2(de, dn))
    return destination(ra, dec, bearing, dist)


def _children(seed: int, k: int):
    ss = np.random.SeedSequence(seed)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(k)]


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

def cfg1_patch(seed: int = SEED_BASE + 1, nA: int = 10_000, n_copies: int = 7_000,
               n_rand: int = 3_000, radius_arcsec: float = 1.0,
               sigma_arcsec: float = 0.3) -> Catalogues:
    """A: nA area-uniform in RA [10, 11), Dec [20, 21). B: n_copies jittered
    copies of distinct A rows plus n_rand uniform in the patch, shuffled."""
    gA, gpar, gjit, grand, _, _ = _children(seed, 6)
    raA, decA = area_uniform(gA, nA, 10.0, 11.0, 20.0, 21.0)
    parents = gpar.choice(nA, size=n_copies, replace=False)
    rj, dj = jitter(gjit, raA[parents], decA[parents], sigma_arcsec)
    rr, dr = area_uniform(grand, n_rand, 10.0, 11.0, 20.0, 21.0)
    raB = np.concatenate([rj, rr])
    decB = np.concatenate([dj, dr])
    perm = gpar.permutation(raB.shape[0])
    return Catalogues("cfg1_patch_10k", raA, decA, raB[perm], decB[perm],
                      radius_arcsec=radius_arcsec,
                      meta=dict(seed=seed, sigma_arcsec=sigma_arcsec))


def _cfg2_mixture(rng: np.random.Generator, n: int, scale: float):
    """The 0.8 / 0.1 / 0.1 mixture: full sphere, cap P1 (RA 0, Dec +10,
    rho 0.5 deg, straddles RA 0/360), cap P2 (RA 0, Dec +89.5, rho 1 deg,
    contains the north pole)."""
    n1 = int(round(0.1 * n))
    n2 = int(round(0.1 * n))
    n0 = n - n1 - n2
    r0, d0 = sphere_uniform(rng, n0)
    r1, d1 = cap_uniform(rng, n1, 0.0, 10.0, 0.5)
    r2, d2 = cap_uniform(rng, n2, 0.0, 89.5, 1.0)
    return np.concatenate([r0, r1, r2]), np.concatenate([d0, d1, d2])


def cfg2_fullsky(scale: float = 1.0, seed: int = SEED_BASE + 2,
                 radius_arcsec: float = 2.0, sigma_arcsec: float = 0.5) -> Catalogues:
    """10M A (8M sphere + 1M in each dense cap) and 10M B (6M jittered copies
    of distinct A rows + 4M random from the same mixture), r = 2"."""
    n = int(round(10_000_000 * scale))
    gA, gpar, gjit, grand, _, _ = _children(seed, 6)
    raA, decA = _cfg2_mixture(gA, n, scale)
    permA = gA.permutation(n)
    raA, decA = raA[permA], decA[permA]
    n_copies = int(round(0.6 * n))
    parents = gpar.choice(n, size=n_copies, replace=False)
    rj, dj = jitter(gjit, raA[parents], decA[parents], sigma_arcsec)
    rr, dr = _cfg2_mixture(grand, n - n_copies, scale)
    raB = np.concatenate([rj, rr])
    decB = np.concatenate([dj, dr])
    perm = gpar.permutation(n)
    return Catalogues(f"cfg2_fullsky_{n}", raA, decA, raB[perm], decB[perm],
                      radius_arcsec=radius_arcsec,
                      meta=dict(seed=seed, scale=scale, sigma_arcsec=sigma_arcsec))


def cfg3_galactic_ellipses(scale: float = 1.0, seed: int = SEED_BASE + 3,
                           nA: int = 100_000, nB: int = 50_000_000,
                           l_hi: float = 60.0) -> Catalogues:
    """Galactic frame. A: clumps with l ~ U[0, l_hi), b area-uniform in
    (-1, 1) deg, semi-major lognormal (median 20", sigma_ln 0.6) resampled
    into [5", 60"], axis ratio U(0.3, 1), PA U(0, 180). B: point sources with
    l ~ U[0, l_hi) and |b| exponential (scale 0.3 deg) truncated at 1 deg.

    ``scale`` shrinks both counts and the longitude range together, so the
    densities (and so the matches per clump) stay those of the full config."""
    nA = max(1, int(round(nA * scale)))
    nB = max(1, int(round(nB * scale)))
    l_hi = l_hi * scale if scale < 1.0 else l_hi
    gA, _, _, grand, garea, _ = _children(seed, 6)
    lA, bA = area_uniform(gA, nA, 0.0, l_hi, -1.0, 1.0)
    a = np.empty(nA)
    todo = np.arange(nA)
    while todo.size:
        v = np.exp(math.log(20.0) + 0.6 * garea.normal(size=todo.size))
        ok = (v >= 5.0) & (v <= 60.0)
        a[todo[ok]] = v[ok]
        todo = todo[~ok]
    q = garea.uniform(0.3, 1.0, nA)
    b = q * a
    pa = garea.uniform(0.0, 180.0, nA)
    lB = grand.uniform(0.0, l_hi, nB)
    u = grand.uniform(0.0, 1.0, nB)
    # inverse CDF of an exponential (scale 0.3) truncated at 1 deg
    absb = -0.3 * np.log1p(-u * (1.0 - math.exp(-1.0 / 0.3)))
    sign = np.where(grand.uniform(size=nB) < 0.5, -1.0, 1.0)
    bB = np.clip(absb * sign, -90.0, 90.0)
    return Catalogues(f"cfg3_galactic_{nA}x{nB}", _norm_ra(lA), bA, _norm_ra(lB), bB,
                      frame=1, shape=1, a_arcsec=a, b_arcsec=b, pa_deg=pa,
                      meta=dict(seed=seed, scale=scale, l_hi=l_hi))


def cfg4_jobs(scale: float = 1.0, seed: int = SEED_BASE + 4, n_jobs: int = 4096,
              max_nA: int = 200_000) -> Catalogues:
    """n_jobs independent circular cross-matches. nA_j lognormal (median 2000,
    sigma_ln 1.0) resampled into [100, 200k] (times ``scale``), nB_j = 10 nA_j;
    each job on its own 0.5 deg cap (centre area-uniform on the sphere); A
    area-uniform in the cap; B = 0.5 nA_j jittered copies (sigma 0.3") plus
    the rest uniform in the cap; radius U[0.5", 10")."""
    gA, gpar, gjit, grand, _, gjob = _children(seed, 6)
    n_jobs = max(1, int(round(n_jobs * min(1.0, scale))))
    nA = np.empty(n_jobs, dtype=np.int64)
    todo = np.arange(n_jobs)
    while todo.size:
        v = np.round(np.exp(math.log(2000.0) + 1.0 * gjob.normal(size=todo.size)))
        ok = (v >= 100) & (v <= max_nA)
        nA[todo[ok]] = v[ok]
        todo = todo[~ok]
    if scale < 1.0:
        nA = np.maximum(1, np.round(nA * scale)).astype(np.int64)
    nB = 10 * nA
    rc, dc = sphere_uniform(gjob, n_jobs)
    radius = gjob.uniform(0.5, 10.0, n_jobs)
    raA, decA, raB, decB = [], [], [], []
    for j in range(n_jobs):
        ra, de = cap_uniform(gA, int(nA[j]), rc[j], dc[j], 0.5)
        nc = int(nA[j] // 2)
        par = gpar.choice(int(nA[j]), size=nc, replace=False)
        rj, dj = jitter(gjit, ra[par], de[par], 0.3)
        rr, dr = cap_uniform(grand, int(nB[j]) - nc, rc[j], dc[j], 0.5)
        rb = np.concatenate([rj, rr])
        db = np.concatenate([dj, dr])
        perm = gpar.permutation(rb.shape[0])
        raA.append(ra)
        decA.append(de)
        raB.append(rb[perm])
        decB.append(db[perm])
    a_off = np.concatenate([[0], np.cumsum(nA)[:-1]])
    b_off = np.concatenate([[0], np.cumsum(nB)[:-1]])
    jobs = np.stack([a_off, nA, b_off, nB, radius], axis=1).astype(np.float64)
    return Catalogues(f"cfg4_jobs_{n_jobs}", np.concatenate(raA), np.concatenate(decA),
                      np.concatenate(raB), np.concatenate(decB), jobs=jobs,
                      meta=dict(seed=seed, scale=scale, n_jobs=n_jobs))


# IAU galactic pole (J2000) — only shapes the synthetic density.
_RA_NGP, _DEC_NGP, _L_NCP = 192.85948, 27.12825, 122.93192


def _gal_to_eq(l: np.ndarray, b: np.ndarray):
    lr, br = l * D2R, b * D2R
    dn = _DEC_NGP * D2R
    dl = (_L_NCP - l) * D2R
    sd = math.sin(dn) * np.sin(br) + math.cos(dn) * np.cos(br) * np.cos(dl)
    y = np.cos(br) * np.sin(dl)
    x = math.cos(dn) * np.sin(br) - math.sin(dn) * np.cos(br) * np.cos(dl)
    ra = _RA_NGP + np.degrees(np.arctan2(y, x))
    dec = np.degrees(np.arcsin(np.clip(sd, -1.0, 1.0)))
    del lr
    return _norm_ra(ra), np.clip(dec, -90.0, 90.0)


_BETA = 5.0 * D2R  # scale height of the galactic-plane term (radians)
_KB = 1.0 / _BETA
# solid-angle weights of the two terms of 1 + 20 exp(-|b| / beta):
# integral of cos b over the sphere, and 20 x that of exp(-|b| / beta) cos b
_W_UNI = 4.0 * math.pi
_W_PLANE = 20.0 * 2.0 * math.pi * 2.0 * (_KB + math.exp(-_KB * math.pi / 2)) / (_KB * _KB + 1.0)


def _plane_clustered(rng: np.random.Generator, n: int):
    """Density (per solid angle) proportional to 1 + 20 exp(-|b| / 5 deg),
    rotated to equatorial. Drawn as the mixture of its two terms: with
    probability W_UNI / (W_UNI + W_PLANE) area-uniform on the sphere, else l
    uniform and |b| with density exp(-|b| / beta) cos b on [0, 90 deg]
    (truncated exponential proposal, accepted with probability cos b), random
    sign."""
    uni = rng.uniform(size=n) < _W_UNI / (_W_UNI + _W_PLANE)
    nu = int(uni.sum())
    lu, bu = sphere_uniform(rng, nu)
    npl = n - nu
    bp = np.empty(0)
    cut = 1.0 - math.exp(-_KB * math.pi / 2)
    while bp.shape[0] < npl:
        m = int((npl - bp.shape[0]) * 1.05) + 64
        t = -_BETA * np.log1p(-rng.uniform(size=m) * cut)
        t = t[rng.uniform(size=m) < np.cos(t)]
        bp = np.concatenate([bp, t])
    bp = np.degrees(bp[:npl]) * np.where(rng.uniform(size=npl) < 0.5, -1.0, 1.0)
    lp = rng.uniform(0.0, 360.0, npl)
    l = np.empty(n)
    b = np.empty(n)
    l[uni], b[uni] = lu, bu
    l[~uni], b[~uni] = lp, np.clip(bp, -90.0, 90.0)
    return _gal_to_eq(l, b)


_PIECE = 4_000_000  # rows per independently seeded piece of a large draw


def _pieces(seed_seq: np.random.SeedSequence, n: int, make, workers: int):
    """Rows 0..n-1 drawn in pieces of _PIECE rows, piece k from its own
    child generator of seed_seq (so the draw does not depend on the number of
    threads), concatenated in piece order. make(rng, lo, hi) returns the
    (ra, dec) of rows [lo, hi)."""
    import concurrent.futures as cf
    bounds = [(lo, min(n, lo + _PIECE)) for lo in range(0, n, _PIECE)]
    kids = seed_seq.spawn(len(bounds))
    gens = [np.random.Generator(np.random.PCG64(k)) for k in kids]
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        parts = list(ex.map(lambda q: make(gens[q], *bounds[q]), range(len(bounds))))
    if not parts:
        return np.zeros(0), np.zeros(0)
    return (np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts]))


def cfg5_scale(scale: float = 1.0, seed: int = SEED_BASE + 5, radius_arcsec: float = 1.5,
               sigma_arcsec: float = 0.4, workers: int = 0) -> Catalogues:
    """200M A with galactic-plane clustering; B = 100M jittered copies of
    distinct A rows + 100M random from the same density; r = 1.5".

    A's rows are independent draws, so its first n/2 rows are a uniformly
    random set of distinct parents for the jittered copies; B is then
    shuffled. Drawn in independently seeded pieces on `workers` threads
    (0: up to 16), with the same result for any thread count."""
    import os
    workers = workers or min(16, os.cpu_count() or 1)
    n = int(round(200_000_000 * scale))
    nc = n // 2
    sA, sjit, srand, sperm = np.random.SeedSequence(seed).spawn(4)
    raA, decA = _pieces(sA, n, lambda g, lo, hi: _plane_clustered(g, hi - lo), workers)
    rj, dj = _pieces(sjit, nc, lambda g, lo, hi: jitter(g, raA[lo:hi], decA[lo:hi],
                                                          sigma_arcsec), workers)
    rr, dr = _pieces(srand, n - nc, lambda g, lo, hi: _plane_clustered(g, hi - lo), workers)
    raB = np.concatenate([rj, rr])
    decB = np.concatenate([dj, dr])
    del rj, dj, rr, dr
    perm = np.random.Generator(np.random.PCG64(sperm)).permutation(n)
    return Catalogues(f"cfg5_scale_{n}", raA, decA, raB[perm], decB[perm],
                      radius_arcsec=radius_arcsec,
                      meta=dict(seed=seed, scale=scale, sigma_arcsec=sigma_arcsec))


def adversarial_circle(seed: int = SEED_BASE + 99, radius_arcsec: float = 1.0,
                       n_centres: int = 64) -> Catalogues:
    """Small catalogue built to stress boundary handling: centres near the
    poles and straddling RA = 0/360, with B placed at distance
    r * (1 +- 2^-45), r * (1 +- 2^-30) and exactly on meridians/parallels.
    Positions are drawn with float64 destination formulas, so the pairs land
    within a few ulps of the boundary; which side each falls on is for the
    oracle to decide."""
    g, = _children(seed, 1)
    dec_c = np.concatenate([
        g.uniform(-89.9999, 89.9999, n_centres // 2),
        np.array([90.0 - 1e-4, -90.0 + 1e-4, 89.99999, 0.0, 45.0, -45.0]),
        g.uniform(88.0, 90.0, n_centres // 4),
    ])
    ra_c = np.concatenate([
        g.uniform(0.0, 360.0, n_centres // 2),
        np.array([0.0, 359.9999999, 180.0, 359.99995, 0.00001, 90.0]),
        g.uniform(0.0, 360.0, n_centres // 4),
    ])
    rad = radius_arcsec * ARCSEC
    pts_r, pts_d = [], []
    for f in (1 - 2.0 ** -45, 1 + 2.0 ** -45, 1 - 2.0 ** -30, 1 + 2.0 ** -30, 1.0, 0.5, 2.0):
        bearings = g.uniform(0.0, 360.0, ra_c.shape[0])
        r, d = destination(ra_c, dec_c, bearings, np.full(ra_c.shape[0], rad * f))
        pts_r.append(r)
        pts_d.append(d)
    raB = np.concatenate(pts_r)
    decB = np.concatenate(pts_d)
    return Catalogues("adversarial_circle", ra_c, dec_c, raB, decB,
                      radius_arcsec=radius_arcsec, meta=dict(seed=seed))
