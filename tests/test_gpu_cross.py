"""GPU parity of c3x_cross_match, the index build over catalogue B and the
match of catalogue A in one call (A keyed and sorted on a second stream
while B's index is built): the oracle's answer for circles, ellipses and
rectangles in both precisions; the same bytes as c3x_build_index followed
by c3x_match, and a kept index that serves later matches; A in the other
frame; one-sweep sorts forced to give up (the call redone one step after the
other); empty catalogues; bad rows of either catalogue."""
import numpy as np
import pytest

import synth
from test_gpu_parity import _t, assert_parity, oracle_match

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


def _area(c3x, cat, dev):
    if cat.shape in (1, 2):
        return dict(shape=cat.shape, a=_t(cat.a_arcsec, dev), b=_t(cat.b_arcsec, dev),
                    pa=_t(cat.pa_deg, dev), pa_zero_deg=cat.pa_zero_deg, pa_sense=cat.pa_sense)
    return dict(shape=0, radius_arcsec=cat.radius_arcsec)


def _cross(c3x, dev, cat, precision, **kw):
    print(f"[gpu] cross {cat.name} precision={precision}", flush=True)
    r = c3x.cross_match(_t(cat.raB, dev), _t(cat.decB, dev), _t(cat.raA, dev), _t(cat.decA, dev),
                        frame=cat.frame, reach_hint_arcsec=cat.reach_arcsec(),
                        precision=precision, **_area(c3x, cat, dev), **kw)
    return r


def _np(r):
    return dict(ia=r.idxA.cpu().numpy(), ib=r.idxB.cpu().numpy(), sep=r.sep.cpu().numpy(),
                best=r.best_idx.cpu().numpy(), best_sep=r.best_sep.cpu().numpy(), stats=r.stats)


def _bytes(r):
    return [t.cpu().numpy().tobytes() for t in (r.idxA, r.idxB, r.sep, r.best_idx, r.best_sep)]


_CASES = {}


def _case(name):
    if name not in _CASES:
        if name == "cfg1":
            cat = synth.cfg1_patch()
        elif name == "cfg2":
            cat = synth.cfg2_fullsky(scale=0.002)
        else:
            cat = synth.cfg3_galactic_ellipses(scale=0.002)
            cat.shape = 1 if name == "ellipse" else 2
        _CASES[name] = (cat, oracle_match(cat))
    return _CASES[name]


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("name", ["cfg1", "cfg2", "ellipse", "rect"])
def test_cross_match_equals_oracle(c3x, dev, name, precision):
    cat, o = _case(name)
    assert len(o.ia) > 1000
    assert_parity(_np(_cross(c3x, dev, cat, precision)), o)


@pytest.mark.parametrize("precision", [0, 1])
def test_same_bytes_as_two_calls_and_kept_index(c3x, dev, precision):
    cat, _ = _case("cfg2")
    r, ix = _cross(c3x, dev, cat, precision, keep_index=True)
    ix2 = c3x.build_index(_t(cat.raB, dev), _t(cat.decB, dev), frame=cat.frame,
                          reach_hint_arcsec=cat.reach_arcsec(), precision=precision)
    r2 = c3x.match(ix2, _t(cat.raA, dev), _t(cat.decA, dev), frame=cat.frame,
                   **_area(c3x, cat, dev))
    assert _bytes(r) == _bytes(r2)
    r3 = c3x.match(ix, _t(cat.raA, dev), _t(cat.decA, dev), frame=cat.frame,
                   **_area(c3x, cat, dev))
    assert _bytes(r3) == _bytes(r2)
    assert ix.stats()["n_cells"] == ix2.stats()["n_cells"]
    ix.free()
    ix2.free()


@pytest.mark.parametrize("precision", [0, 1])
def test_catalogue_a_in_the_other_frame(c3x, dev, precision):
    from oracle import frames
    g = np.random.default_rng(21)
    raA, decA = synth.cap_uniform(g, 20_000, 305.0, 40.0, 0.5)
    rb, db = synth.cap_uniform(g, 40_000, 305.0, 40.0, 0.5)
    rB, dB, _ = frames.convert(rb, db, 0, 1)
    a = g.uniform(5.0, 40.0, 20_000)
    kw = dict(a=a, b=a * g.uniform(0.3, 1.0, 20_000), pa=g.uniform(0, 180, 20_000),
              pa_zero_deg=15.0, pa_sense=-1)
    o = frames.match_mixed(raA, decA, 0, rB, dB, 1, shape=1, **kw)
    assert len(o.ia) > 5000
    print(f"[gpu] cross across frames precision={precision}", flush=True)
    r = c3x.cross_match(_t(rB, dev), _t(dB, dev), _t(raA, dev), _t(decA, dev), frame=1,
                        frameA=0, reach_hint_arcsec=float(a.max()), precision=precision,
                        shape=1, a=_t(kw["a"], dev), b=_t(kw["b"], dev), pa=_t(kw["pa"], dev),
                        pa_zero_deg=15.0, pa_sense=-1)
    assert_parity(_np(r), o)


@pytest.mark.parametrize("precision", [0, 1])
def test_one_sweep_give_up_is_redone(c3x, dev, precision, monkeypatch):
    """Every sort takes the one-sweep schedule and every look-back gives up at
    once (its slots poisoned): the call is redone one step after the other,
    with the table schedule, and returns the oracle's answer."""
    cat, o = _case("cfg2")
    monkeypatch.setenv("C3X_DEBUG_ONESWEEP_TILES", "1")
    monkeypatch.setenv("C3X_DEBUG_SORT_SPIN", "0")
    r = _np(_cross(c3x, dev, cat, precision))
    assert_parity(r, o)
    assert r["stats"]["n_sort_retries"] == 1


def test_on_a_caller_stream(c3x, dev):
    """On a stream of the caller's (the second stream waits for the grid
    uploaded on it): the same bytes as on the null stream."""
    import torch
    cat, _ = _case("cfg1")
    want = _bytes(_cross(c3x, dev, cat, 1))
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        tens = [_t(x, dev) for x in (cat.raB, cat.decB, cat.raA, cat.decA)]
        r = c3x.cross_match(*tens, reach_hint_arcsec=cat.reach_arcsec(), precision=1,
                            radius_arcsec=cat.radius_arcsec, stream=st)
    st.synchronize()
    assert _bytes(r) == want


def test_empty_catalogues(c3x, dev):
    cat, _ = _case("cfg1")
    e = np.zeros(0)
    for ra, de, rb, db in ((e, e, cat.raB, cat.decB), (cat.raA, cat.decA, e, e), (e, e, e, e)):
        r = c3x.cross_match(_t(rb, dev), _t(db, dev), _t(ra, dev), _t(de, dev),
                            reach_hint_arcsec=2.0, radius_arcsec=2.0)
        assert r.n_pairs == 0
        assert r.best_idx.shape[0] == len(ra)
        assert bool((r.best_idx == -1).all())


def test_bad_rows(c3x, dev):
    cat, _ = _case("cfg1")
    rb = cat.raB.copy()
    rb[7] = 361.0
    with pytest.raises(c3x.C3XError) as ei:
        c3x.cross_match(_t(rb, dev), _t(cat.decB, dev), _t(cat.raA, dev), _t(cat.decA, dev),
                        reach_hint_arcsec=2.0)
    assert "catalogue B row 7" in str(ei.value)
    da = cat.decA.copy()
    da[3] = float("nan")
    with pytest.raises(c3x.C3XError) as ei:
        c3x.cross_match(_t(cat.raB, dev), _t(cat.decB, dev), _t(cat.raA, dev), _t(da, dev),
                        reach_hint_arcsec=2.0)
    assert "catalogue A row 3" in str(ei.value)
