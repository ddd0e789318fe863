"""GPU parity of the Exact Value case (c3x_exact_match; paper Section 2.1,
rows match when their chosen columns hold equal values, with Section 2.2's
all and best selections and join types) against oracle/exact_value.py:
identical pairs and best matches, bit for bit. Cases: the hand-worked
example (int64 extremes, +0 / -0, NaN), random columns with heavy
duplication and a skewed value (one value held by thousands of rows),
BEST-only output, empty inputs, the join types through
c3x_result_unmatched, and a 2M x 2M draw."""
import json
import os

import numpy as np
import pytest

from oracle import exact_value, join

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def c3x(dev):
    import paper_1611_08494_amd as m
    m.lib()
    return m


def _check(c3x, dev, vA, vB, kind, mode=3):
    import torch
    print(f"[gpu] exact value {kind} {len(vA)} x {len(vB)} mode={mode}", flush=True)
    dt = torch.int64 if kind == "i64" else torch.float64
    tA = torch.as_tensor(vA, dtype=dt, device=dev)
    tB = torch.as_tensor(vB, dtype=dt, device=dev)
    r = c3x.exact_match(tA, tB, mode=mode)
    ia, ib, best = exact_value.match(vA, vB, kind)
    g_best = r.best_idx.cpu().numpy()
    assert np.array_equal(g_best, best)
    if mode & 1:
        assert np.array_equal(r.idxA.cpu().numpy(), ia)
        assert np.array_equal(r.idxB.cpu().numpy(), ib)
        assert np.all(r.sep.cpu().numpy() == 0.0)
    else:
        m = best >= 0
        assert np.array_equal(r.idxA.cpu().numpy(), np.nonzero(m)[0])
        assert np.array_equal(r.idxB.cpu().numpy(), best[m])
    bs = r.best_sep.cpu().numpy()
    assert np.all(bs[best >= 0] == 0.0) and np.all(np.isnan(bs[best < 0]))
    return r, ia, ib, best


@pytest.mark.parametrize("kind", ["i64", "f64"])
def test_hand_example(c3x, dev, kind):
    ex = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                     "exact_value_example.json")))[kind]
    conv = (lambda v: np.array(v, dtype=np.int64)) if kind == "i64" else \
        (lambda v: np.array([float(x) for x in v]))
    for mode in (1, 2, 3):
        _check(c3x, dev, conv(ex["A"]), conv(ex["B"]), kind, mode)


@pytest.mark.parametrize("kind", ["i64", "f64"])
def test_duplicates_and_skew(c3x, dev, kind):
    g = np.random.default_rng(8)
    vA = g.integers(0, 30_000, 60_000)
    vB = g.integers(0, 30_000, 90_000)
    vA[:3000] = 77  # one value held by thousands of rows on both sides
    vB[-2000:] = 77
    if kind == "f64":
        vA = vA * 0.5 - 100.0
        vB = vB * 0.5 - 100.0
        vA[5:9] = [np.nan, -0.0, 0.0, np.inf]
        vB[7:11] = [np.nan, 0.0, -0.0, np.inf]
    else:
        vA = vA.astype(np.int64) - 12345
        vB = vB.astype(np.int64) - 12345
    r, ia, ib, best = _check(c3x, dev, vA, vB, kind)
    assert len(ia) > 6_000_000
    _check(c3x, dev, vA, vB, kind, mode=2)
    # join types: the rows in no stored pair
    for sel, name in ((c3x.ALL, "all"), (c3x.BEST, "best")):
        ua, ub = c3x.unmatched(r, sel)
        pa, pb = join.stored_pairs(ia, ib, best, name)
        wa, wb = join.unmatched(len(vA), len(vB), pa, pb)
        assert np.array_equal(ua.cpu().numpy(), wa) and np.array_equal(ub.cpu().numpy(), wb)


def test_empty_and_large(c3x, dev):
    e = np.zeros(0, dtype=np.int64)
    one = np.array([5], dtype=np.int64)
    for a, b in ((e, one), (one, e), (e, e)):
        _check(c3x, dev, a, b, "i64")
    g = np.random.default_rng(9)
    vA = g.integers(0, 3_000_000, 2_000_000).astype(np.int64)
    vB = g.integers(0, 3_000_000, 2_000_000).astype(np.int64)
    _check(c3x, dev, vA, vB, "i64")
