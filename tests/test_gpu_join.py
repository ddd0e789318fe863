"""GPU parity of the join types (Section 2.2, "Match selection and join
types"): the unmatched rows c3x_result_unmatched finds (through the C ABI)
against the oracle's, exactly, for both selections and both precisions, on
the 10k x 10k patch, a scaled full-sky draw (several 4096-row tiles and a
ragged tail) and the full 10M x 10M full-sky workload; every join type
assembled from them; empty catalogues and the error cases."""
import numpy as np
import pytest

import synth

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


def _t(x, dev):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64), device=dev)


def _match(c3x, dev, cat, precision, mode):
    print(f"[gpu] {cat.name} precision={precision} mode={mode}", flush=True)
    ix = c3x.build_index(_t(cat.raB, dev), _t(cat.decB, dev), reach_hint_arcsec=cat.radius_arcsec,
                         precision=precision)
    r = c3x.match(ix, _t(cat.raA, dev), _t(cat.decA, dev), mode=mode,
                  radius_arcsec=cat.radius_arcsec)
    ix.free()
    return r


def _oracle(cat):
    import oracle
    return oracle.match(cat.raA, cat.decA, cat.raB, cat.decB, radius_arcsec=cat.radius_arcsec)


def _expected(cat, o, selection):
    from oracle import join as J
    pa, pb = J.stored_pairs(o.ia, o.ib, o.best_idx, selection)
    return J.unmatched(cat.nA, cat.nB, pa, pb)


@pytest.fixture(scope="module")
def cfg1():
    cat = synth.cfg1_patch()
    return cat, _oracle(cat)


@pytest.fixture(scope="module")
def fullsky_small():
    cat = synth.cfg2_fullsky(scale=0.002)
    return cat, _oracle(cat)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("selection", ["all", "best"])
@pytest.mark.parametrize("which", ["cfg1", "fullsky_small"])
def test_unmatched_rows_match_oracle(c3x, dev, request, precision, selection, which):
    cat, o = request.getfixturevalue(which)
    r = _match(c3x, dev, cat, precision, c3x.ALL | c3x.BEST)
    ua, ub = c3x.unmatched(r, c3x.ALL if selection == "all" else c3x.BEST)
    wa, wb = _expected(cat, o, selection)
    assert np.array_equal(ua.cpu().numpy(), wa)
    assert np.array_equal(ub.cpu().numpy(), wb)
    assert 0 < len(wa) < cat.nA and 0 < len(wb) < cat.nB


@pytest.mark.parametrize("how", ["1and2", "1or2", "all1", "all2", "1not2", "2not1", "1xor2"])
def test_join_types_match_oracle(c3x, dev, cfg1, how):
    from oracle import join as J
    cat, o = cfg1
    r = _match(c3x, dev, cat, 1, c3x.ALL | c3x.BEST)
    for sel, selname in ((c3x.ALL, "all"), (c3x.BEST, "best")):
        got = c3x.join(r, how, selection=sel)
        pa, pb = J.stored_pairs(o.ia, o.ib, o.best_idx, selname)
        wpa, wpb, wa, wb = J.join(cat.nA, cat.nB, pa, pb, how)
        if sel == c3x.ALL and len(wpa):
            assert np.array_equal(got["idxA"].cpu().numpy(), wpa)
            assert np.array_equal(got["idxB"].cpu().numpy(), wpb)
        elif sel == c3x.BEST and len(wpa):
            best = got["best_idx"].cpu().numpy()
            rows = np.nonzero(best >= 0)[0]
            assert np.array_equal(rows, wpa) and np.array_equal(best[rows], wpb)
        else:
            assert got["idxA"] is None and got["best_idx"] is None
        for key, want in (("rowsA", wa), ("rowsB", wb)):
            if got[key] is None:
                assert len(want) == 0
            else:
                assert np.array_equal(got[key].cpu().numpy(), want)


def test_best_only_result(c3x, dev, cfg1):
    """A best-only result: selection BEST works, ALL is refused; a repeat
    gives the same rows."""
    cat, o = cfg1
    r = _match(c3x, dev, cat, 0, c3x.BEST)
    wa, wb = _expected(cat, o, "best")
    for _ in range(2):
        ua, ub = c3x.unmatched(r, c3x.BEST)
        assert np.array_equal(ua.cpu().numpy(), wa)
        assert np.array_equal(ub.cpu().numpy(), wb)
    with pytest.raises(c3x.C3XError, match="C3X_ALL"):
        c3x.unmatched(r, c3x.ALL)
    r2 = _match(c3x, dev, cat, 0, c3x.ALL)
    with pytest.raises(c3x.C3XError, match="C3X_BEST"):
        c3x.unmatched(r2, c3x.BEST)
    with pytest.raises(c3x.C3XError, match="selection"):
        c3x.unmatched(r2, 0)


@pytest.mark.parametrize("precision", [0, 1])
def test_empty_catalogues(c3x, dev, precision):
    e = np.zeros(0)
    pts = np.array([10.0, 20.0, 30.0])
    for ra_a, ra_b in ((e, pts), (pts, e), (e, e)):
        cat = synth.Catalogues("empty", ra_a, ra_a * 0, ra_b, ra_b * 0, radius_arcsec=1.0)
        r = _match(c3x, dev, cat, precision, c3x.ALL | c3x.BEST)
        for sel in (c3x.ALL, c3x.BEST):
            ua, ub = c3x.unmatched(r, sel)
            assert ua.cpu().numpy().tolist() == list(range(len(ra_a)))
            assert ub.cpu().numpy().tolist() == list(range(len(ra_b)))


def test_batch_result_is_refused(c3x, dev):
    ra = _t([10.0, 10.0], dev)
    de = _t([0.0, 0.0], dev)
    b = c3x.Batch([(0, 1, 0, 1, 1.0), (1, 1, 1, 1, 1.0)], ra, de, ra, de, precision=0)
    with pytest.raises(c3x.C3XError, match="batch"):
        c3x.unmatched(b.result(), c3x.ALL)
    b.free()


@pytest.mark.slow
def test_full_size_fullsky(c3x, dev):
    """The 10M x 10M full-sky workload of the benchmark, both selections,
    against the oracle's whole result."""
    cat = synth.cfg2_fullsky(scale=1.0)
    o = _oracle(cat)
    r = _match(c3x, dev, cat, 1, c3x.ALL | c3x.BEST)
    for sel, name in ((c3x.ALL, "all"), (c3x.BEST, "best")):
        ua, ub = c3x.unmatched(r, sel)
        wa, wb = _expected(cat, o, name)
        assert np.array_equal(ua.cpu().numpy(), wa)
        assert np.array_equal(ub.cpu().numpy(), wb)
