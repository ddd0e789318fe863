"""Pins for the oracle's symmetric best pairs (oracle/mutual.py; paper
Section 2.2, the "best" match selection read as pairs that are each other's
nearest match):

* a hand-worked example with exact separations and ties on both sides
  (tests/golden/mutual_example.json);
* the definition restated as loops over 200-bit angles on tiny random
  catalogues (every pair decided and ranked in mpmath, no FP64 ladder);
* invariants: circle symmetry (the pairs of A against B are those of B
  against A, transposed), one pair per row at most, a subset of the best
  matches.
"""
import json
import os

import numpy as np
import pytest

import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "mutual_example.json")


def _mutual(o, c, nB):
    from oracle import mutual
    return mutual.mutual(c["raA"], c["decA"], c["raB"], c["decB"], o.ia, o.ib, o.sep,
                         o.best_idx, nB)


def test_hand_example(oracle_lib):
    ex = json.load(open(GOLD))
    c = {k: np.array(ex[k]) for k in ("raA", "decA", "raB", "decB")}
    o = oracle_lib.match(c["raA"], c["decA"], c["raB"], c["decB"],
                         radius_arcsec=ex["radius_arcsec"])
    assert o.best_idx.tolist() == ex["best"]
    pa, pb, ps, bb = _mutual(o, c, len(ex["raB"]))
    assert bb.tolist() == ex["best_b"]
    assert pa.tolist() == ex["mutual_a"] and pb.tolist() == ex["mutual_b"]
    d = 2.0 ** -12 * 3600
    assert np.allclose(ps, [d, d, 0.5 * d], rtol=0, atol=1e-9)


def _definition(raA, decA, raB, decB, radius):
    """Symmetric best pairs straight from the definition: every pair decided
    and every angle taken at 200 bits, minima by (theta, row) in loops."""
    from oracle import exact
    nA, nB = len(raA), len(raB)
    th = {}
    for i in range(nA):
        for j in range(nB):
            if exact.decide_circle(raA[i], decA[i], raB[j], decB[j], radius):
                th[(i, j)] = exact.theta(raA[i], decA[i], raB[j], decB[j])

    import mpmath

    def argmin(cands):
        best = None
        with mpmath.workprec(exact.PREC_BITS):
            for t, r in sorted(cands, key=lambda x: x[1]):
                if best is None or t < best[0] * (1 - exact.TIE_REL):
                    best = (t, r)
        return -1 if best is None else best[1]

    bA = [argmin([(t, j) for (i, j), t in th.items() if i == a]) for a in range(nA)]
    bB = [argmin([(t, i) for (i, j), t in th.items() if j == b]) for b in range(nB)]
    pairs = [(a, bA[a]) for a in range(nA) if bA[a] >= 0 and bB[bA[a]] == a]
    return bA, bB, pairs


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_against_definition_200_bit(oracle_lib, seed):
    g = np.random.default_rng(seed)
    # clustered so that rows have several matches, with exact duplicates
    raA, decA = synth.cap_uniform(g, 14, 123.0, 88.5 if seed == 3 else -20.0, 0.002)
    raB, decB = synth.cap_uniform(g, 18, 123.0, 88.5 if seed == 3 else -20.0, 0.002)
    raB[:2], decB[:2] = raA[:2], decA[:2]
    raB[2], decB[2] = raB[3], decB[3]      # two B rows at one place: ties seen from A
    raA[5], decA[5] = raA[4], decA[4]      # two A rows at one place: ties seen from B
    radius = 5.0
    bA, bB, pairs = _definition(raA, decA, raB, decB, radius)
    assert sum(1 for x in bA if x >= 0) > 5
    o = oracle_lib.match(raA, decA, raB, decB, radius_arcsec=radius)
    assert o.best_idx.tolist() == bA
    c = dict(raA=raA, decA=decA, raB=raB, decB=decB)
    pa, pb, _, bb = _mutual(o, c, len(raB))
    assert bb.tolist() == bB
    assert list(zip(pa.tolist(), pb.tolist())) == pairs


def test_invariants(oracle_lib):
    c = synth.cfg2_fullsky(scale=0.0008)
    r = 40.0
    ab = oracle_lib.match(c.raA, c.decA, c.raB, c.decB, radius_arcsec=r)
    ba = oracle_lib.match(c.raB, c.decB, c.raA, c.decA, radius_arcsec=r)
    da = dict(raA=c.raA, decA=c.decA, raB=c.raB, decB=c.decB)
    db = dict(raA=c.raB, decA=c.decB, raB=c.raA, decB=c.decA)
    pa, pb, ps, _ = _mutual(ab, da, c.nB)
    qa, qb, qs, _ = _mutual(ba, db, c.nA)
    assert len(pa) > 500
    # the circle is symmetric: B-against-A pairs are the A-against-B ones, transposed
    assert sorted(zip(pa.tolist(), pb.tolist())) == sorted(zip(qb.tolist(), qa.tolist()))
    assert len(set(pa.tolist())) == len(pa) and len(set(pb.tolist())) == len(pb)
    assert np.all(ab.best_idx[pa] == pb)
    # fewer symmetric pairs than best matches: some B rows are several rows' best
    assert len(pa) < int((ab.best_idx >= 0).sum())


def test_near_ties_seen_from_b_are_ranked_exactly(oracle_lib):
    """Two A rows on the meridian of one B row: A0 due south at d', A1 due
    north at d, with d' one ulp above d (exact angles |Dec|). Where the FP64
    separations come out equal, only the exact ranking sees that A1, the
    higher row, is nearer; at d' = d (an exact tie) the lower row wins."""
    import math
    from oracle import mutual
    raB, decB = np.array([40.0]), np.array([0.0])
    equal = 0
    for k in range(200):
        d = 2.0 ** -12 * (1.0 + k / 211.0)
        for dp, want in ((math.nextafter(d, 1.0), 1), (d, 0)):
            raA = np.array([40.0, 40.0])
            decA = np.array([-dp, d])
            o = oracle_lib.match(raA, decA, raB, decB, radius_arcsec=30.0)
            assert len(o.ia) == 2
            if dp != d and o.sep[0] == o.sep[1]:
                equal += 1
            bb = mutual.best_of_b(raA, decA, raB, decB, o.ia, o.ib, o.sep, 1)
            assert bb.tolist() == [want], (k, dp, d)
    assert equal >= 5
