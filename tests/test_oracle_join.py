"""Pins of the oracle's join types (Section 2.2, "Match selection and join
types"): a hand-written example, a brute-force restatement on tiny random
inputs, and set identities on a real cross-match."""
import json
import os

import numpy as np
import pytest

from oracle import join as J

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "join_example.json")


def _ex():
    return json.load(open(GOLDEN))


@pytest.mark.parametrize("selection", ["all", "best"])
@pytest.mark.parametrize("how", J.JOINS)
def test_hand_written_example(selection, how):
    ex = _ex()
    ia = np.array([p[0] for p in ex["pairs_all"]], dtype=np.int32)
    ib = np.array([p[1] for p in ex["pairs_all"]], dtype=np.int32)
    pa, pb = J.stored_pairs(ia, ib, np.array(ex["best_idx"]), selection)
    got = J.join(ex["nA"], ex["nB"], pa, pb, how)
    want = ex["expect"][selection][how]
    assert [[int(a), int(b)] for a, b in zip(got[0], got[1])] == want["pairs"]
    assert got[2].tolist() == want["a"]
    assert got[3].tolist() == want["b"]


def _brute(nA, nB, pairs, how):
    """The definitions as loops: a row is unmatched when no pair names it."""
    ua = [a for a in range(nA) if all(p[0] != a for p in pairs)]
    ub = [b for b in range(nB) if all(p[1] != b for p in pairs)]
    keep_p = how in ("1and2", "1or2", "all1", "all2")
    keep_a = how in ("1or2", "all1", "1not2", "1xor2")
    keep_b = how in ("1or2", "all2", "2not1", "1xor2")
    return (pairs if keep_p else []), (ua if keep_a else []), (ub if keep_b else [])


def test_brute_force_tiny():
    rng = np.random.default_rng(7)
    for _ in range(200):
        nA, nB = int(rng.integers(0, 7)), int(rng.integers(0, 7))
        m = int(rng.integers(0, 9)) if nA and nB else 0
        pairs = sorted({(int(rng.integers(0, nA)), int(rng.integers(0, nB))) for _ in range(m)})
        pa = np.array([p[0] for p in pairs], dtype=np.int32)
        pb = np.array([p[1] for p in pairs], dtype=np.int32)
        for how in J.JOINS:
            got = J.join(nA, nB, pa, pb, how)
            want = _brute(nA, nB, pairs, how)
            assert list(zip(got[0].tolist(), got[1].tolist())) == want[0]
            assert got[2].tolist() == want[1]
            assert got[3].tolist() == want[2]


def test_identities_on_a_cross_match():
    """On a real result: every A row is matched or not (exactly once); an A
    row's matchedness does not depend on the selection; best-only stores a
    subset of the pairs, so it leaves at least the same B rows unmatched;
    xor = (1 not 2) + (2 not 1)."""
    import oracle
    import synth
    cat = synth.cfg1_patch(nA=3000, n_copies=2000, n_rand=1000)
    o = oracle.match(cat.raA, cat.decA, cat.raB, cat.decB, radius_arcsec=cat.radius_arcsec)
    ua_all, ub_all = J.unmatched(cat.nA, cat.nB, o.ia, o.ib)
    pa, pb = J.stored_pairs(o.ia, o.ib, o.best_idx, "best")
    ua_best, ub_best = J.unmatched(cat.nA, cat.nB, pa, pb)
    assert len(ua_all) + len(np.unique(o.ia)) == cat.nA
    assert np.array_equal(ua_all, ua_best)
    assert np.array_equal(ua_all, np.nonzero(o.best_idx < 0)[0])
    assert set(ub_all.tolist()) <= set(ub_best.tolist())
    assert len(ub_all) + len(np.unique(o.ib)) == cat.nB
    x = J.join(cat.nA, cat.nB, o.ia, o.ib, "1xor2")
    assert np.array_equal(x[2], J.join(cat.nA, cat.nB, o.ia, o.ib, "1not2")[2])
    assert np.array_equal(x[3], J.join(cat.nA, cat.nB, o.ia, o.ib, "2not1")[3])
    assert 0 < len(ua_all) < cat.nA and 0 < len(ub_all) < cat.nB
