"""Pins for the oracle's Exact Value case (oracle/exact_value.py; paper
Section 2.1, rows match when their chosen columns hold equal values, and
Section 2.2's all / best selections):

* a hand-worked example for int64 and float64 columns (duplicates, the
  int64 extremes, +0 / -0, NaN, neighbouring doubles), in
  tests/golden/exact_value_example.json;
* the definition as an all-pairs comparison (numpy ==) on small random
  columns with many repeated values;
* invariants: swapping the catalogues transposes the pairs; the pair count
  is the sum over values of (A rows) x (B rows) holding it.
"""
import json
import os

import numpy as np
import pytest

from oracle import exact_value

GOLD = os.path.join(os.path.dirname(__file__), "golden", "exact_value_example.json")


def _col(vals, kind):
    if kind == "i64":
        return np.array(vals, dtype=np.int64)
    return np.array([float(v) for v in vals], dtype=np.float64)


@pytest.mark.parametrize("kind", ["i64", "f64"])
def test_hand_example(kind):
    ex = json.load(open(GOLD))[kind]
    ia, ib, best = exact_value.match(_col(ex["A"], kind), _col(ex["B"], kind), kind)
    assert [[int(a), int(b)] for a, b in zip(ia, ib)] == ex["pairs"]
    assert best.tolist() == ex["best"]


def _definition(vA, vB):
    eq = vA[:, None] == vB[None, :]     # numeric ==: +0 == -0, NaN != anything
    ia, ib = np.nonzero(eq)
    best = np.where(eq.any(axis=1), eq.argmax(axis=1), -1)
    return ia, ib, best


@pytest.mark.parametrize("kind", ["i64", "f64"])
@pytest.mark.parametrize("seed", [1, 2])
def test_against_all_pairs(kind, seed):
    g = np.random.default_rng(seed)
    if kind == "i64":
        vA = g.integers(-20, 20, 300).astype(np.int64)
        vB = g.integers(-20, 20, 400).astype(np.int64)
        vA[:3] = [np.iinfo(np.int64).max, np.iinfo(np.int64).min, 0]
        vB[:2] = [np.iinfo(np.int64).max, 5]
    else:
        vA = g.integers(-20, 20, 300) * 0.25
        vB = g.integers(-20, 20, 400) * 0.25
        vA[:4] = [np.nan, -0.0, 0.0, np.nextafter(1.0, 2.0)]
        vB[:4] = [np.nan, 0.0, -0.0, 1.0]
    ia, ib, best = exact_value.match(vA, vB, kind)
    da, db, dbest = _definition(vA, vB)
    assert np.array_equal(ia, da) and np.array_equal(ib, db)
    assert np.array_equal(best, dbest)
    assert len(ia) > 1000


def test_invariants():
    g = np.random.default_rng(3)
    vA = g.integers(0, 50, 500).astype(np.int64)
    vB = g.integers(0, 50, 700).astype(np.int64)
    ia, ib, _ = exact_value.match(vA, vB, "i64")
    ja, jb, _ = exact_value.match(vB, vA, "i64")
    assert sorted(zip(ia.tolist(), ib.tolist())) == sorted(zip(jb.tolist(), ja.tolist()))
    ca, cb = np.bincount(vA, minlength=50), np.bincount(vB, minlength=50)
    assert len(ia) == int((ca * cb).sum())
