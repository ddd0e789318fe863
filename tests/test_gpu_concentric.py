"""GPU parity of the concentric ellipses (Section 3, ClumpPopulator):
c3x_match_concentric through the C ABI against the oracle -- identical
pairs, separations within 1e-6", identical levels and best matches -- on a
scaled galactic-ellipse workload, both precisions; every level decided in
binary128 on the host (a test setting); A in the other frame; the
closed-form axis placements; one scale equal to the plain elliptical match;
empty input and the error cases."""
import json
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

SEP_TOL = 1e-6
SCALES = [0.5, 1.0, 1.5, 2.0]
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "concentric_axes.json")


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


def _run(c3x, dev, cat, precision, scales, mode=None):
    print(f"[gpu] {cat.name} precision={precision} scales={scales}", flush=True)
    ix = c3x.build_index(_t(cat.raB, dev), _t(cat.decB, dev), frame=cat.frame,
                         reach_hint_arcsec=float(np.max(cat.a_arcsec, initial=1.0)) *
                         max(scales, default=1.0),
                         precision=precision)
    r = c3x.match_concentric(ix, _t(cat.raA, dev), _t(cat.decA, dev), _t(cat.a_arcsec, dev),
                             _t(cat.b_arcsec, dev), _t(cat.pa_deg, dev), scales, frame=cat.frame,
                             pa_zero_deg=cat.pa_zero_deg, pa_sense=cat.pa_sense,
                             mode=c3x.ALL | c3x.BEST if mode is None else mode)
    ix.free()
    return r


@pytest.fixture(scope="module")
def ellipses():
    import oracle
    from oracle import concentric as C
    cat = synth.cfg3_galactic_ellipses(scale=0.002)
    kw = dict(pa_zero_deg=cat.pa_zero_deg, pa_sense=cat.pa_sense)
    c = C.concentric(cat.raA, cat.decA, cat.raB, cat.decB, cat.a_arcsec, cat.b_arcsec,
                     cat.pa_deg, SCALES, **kw)
    outer = oracle.match(cat.raA, cat.decA, cat.raB, cat.decB, shape=1,
                         a=cat.a_arcsec * SCALES[-1], b=cat.b_arcsec * SCALES[-1], pa=cat.pa_deg,
                         **kw)
    return cat, c, outer


@pytest.mark.parametrize("precision", [0, 1])
def test_levels_match_oracle(c3x, dev, ellipses, precision):
    cat, c, outer = ellipses
    r = _run(c3x, dev, cat, precision, SCALES)
    assert np.array_equal(r.idxA.cpu().numpy(), c.ia)
    assert np.array_equal(r.idxB.cpu().numpy(), c.ib)
    assert np.abs(r.sep.cpu().numpy() - c.sep).max() <= SEP_TOL
    assert np.array_equal(r.level.cpu().numpy(), c.level)
    assert np.array_equal(r.best_idx.cpu().numpy(), outer.best_idx)
    assert len(np.unique(c.level)) == len(SCALES)


def test_levels_decided_on_the_host(c3x, dev, ellipses, monkeypatch):
    """C3X_DEBUG_FORCE_AMBIG: the FP64 level test decides nothing, so every
    pair with a smaller scale to decide is decided from scale 0 up in
    binary128 on the host; the levels stay the oracle's."""
    cat, c, _ = ellipses
    monkeypatch.setenv("C3X_DEBUG_FORCE_AMBIG", "1")
    for precision in (0, 1):
        r = _run(c3x, dev, cat, precision, SCALES)
        assert np.array_equal(r.idxA.cpu().numpy(), c.ia)
        assert np.array_equal(r.idxB.cpu().numpy(), c.ib)
        assert np.array_equal(r.level.cpu().numpy(), c.level)
        assert r.stats["n_ambiguous"] >= int(np.count_nonzero(c.level > 0))


@pytest.mark.parametrize("precision", [0, 1])
def test_levels_across_frames(c3x, dev, precision):
    """A in the galactic frame against an equatorial index: the oracle's
    levels of A converted by the frame rule (orientations turned by its
    gamma) against the index's B."""
    from oracle import concentric as C
    from oracle import frames
    c = synth.cfg3_galactic_ellipses(scale=0.001)
    gal, eq = 1, 0
    rB, dB, _ = frames.convert(c.raB, c.decB, gal, eq)
    ra2, dec2, gam = frames.convert(c.raA, c.decA, gal, eq)
    T = (c.pa_zero_deg + c.pa_sense * c.pa_deg) + gam
    o = C.concentric(ra2, dec2, rB, dB, c.a_arcsec, c.b_arcsec, T, SCALES)
    assert len(o.ia) > 1000
    print(f"[gpu] concentric across frames precision={precision}", flush=True)
    ix = c3x.build_index(_t(rB, dev), _t(dB, dev), frame=eq,
                         reach_hint_arcsec=float(np.max(c.a_arcsec)) * SCALES[-1],
                         precision=precision)
    r = c3x.match_concentric(ix, _t(c.raA, dev), _t(c.decA, dev), _t(c.a_arcsec, dev),
                             _t(c.b_arcsec, dev), _t(c.pa_deg, dev), SCALES, frame=gal,
                             pa_zero_deg=c.pa_zero_deg, pa_sense=c.pa_sense, mode=c3x.ALL)
    ix.free()
    assert np.array_equal(r.idxA.cpu().numpy(), o.ia)
    assert np.array_equal(r.idxB.cpu().numpy(), o.ib)
    assert np.abs(r.sep.cpu().numpy() - o.sep).max() <= SEP_TOL
    assert np.array_equal(r.level.cpu().numpy(), o.level)


@pytest.mark.parametrize("ci", range(6))
def test_axis_placements(c3x, dev, ci):
    from test_oracle_concentric import axis_catalogue
    ex = json.load(open(GOLDEN))
    case = ex["cases"][ci]
    raA, decA, raB, decB, want = axis_catalogue(ex, case)
    n = raA.size
    cat = synth.Catalogues("axes", raA, decA, raB, decB, shape=1,
                           a_arcsec=np.full(n, ex["a_arcsec"]), b_arcsec=np.full(n, ex["b_arcsec"]),
                           pa_deg=np.full(n, case["pa_deg"]))
    for precision in (0, 1):
        r = _run(c3x, dev, cat, precision, ex["scales"])
        got = list(zip(r.idxA.cpu().numpy().tolist(), r.idxB.cpu().numpy().tolist(),
                       r.level.cpu().numpy().tolist()))
        assert got == want


def test_one_scale_is_the_elliptical_match(c3x, dev, ellipses):
    cat, _, _ = ellipses
    r = _run(c3x, dev, cat, 1, [1.0])
    ix = c3x.build_index(_t(cat.raB, dev), _t(cat.decB, dev), frame=cat.frame,
                         reach_hint_arcsec=60.0, precision=1)
    p = c3x.match(ix, _t(cat.raA, dev), _t(cat.decA, dev), frame=cat.frame, shape=c3x.ELLIPSE,
                  a=_t(cat.a_arcsec, dev), b=_t(cat.b_arcsec, dev), pa=_t(cat.pa_deg, dev),
                  pa_zero_deg=cat.pa_zero_deg, pa_sense=cat.pa_sense)
    ix.free()
    assert np.array_equal(r.idxA.cpu().numpy(), p.idxA.cpu().numpy())
    assert np.array_equal(r.idxB.cpu().numpy(), p.idxB.cpu().numpy())
    assert np.all(r.level.cpu().numpy() == 0)


def test_empty_and_errors(c3x, dev, ellipses):
    cat, _, _ = ellipses
    e = synth.Catalogues("empty", np.zeros(0), np.zeros(0), cat.raB[:10], cat.decB[:10],
                         shape=1, a_arcsec=np.zeros(0), b_arcsec=np.zeros(0), pa_deg=np.zeros(0))
    r = _run(c3x, dev, e, 0, SCALES)
    assert r.n_pairs == 0 and r.level.shape[0] == 0
    for bad in ([1.0, 0.5], [0.0, 1.0], [], [1.0, float("nan")]):
        with pytest.raises(c3x.C3XError, match="scales"):
            _run(c3x, dev, cat, 0, bad)
    with pytest.raises(c3x.C3XError, match="C3X_ALL"):
        _run(c3x, dev, cat, 0, SCALES, mode=c3x.BEST)
    big = synth.Catalogues("big", cat.raA[:5], cat.decA[:5], cat.raB[:10], cat.decB[:10],
                           shape=1, a_arcsec=np.full(5, 200000.0), b_arcsec=np.full(5, 150000.0),
                           pa_deg=np.zeros(5))
    with pytest.raises(c3x.C3XError, match="scale 3"):
        _run(c3x, dev, big, 0, SCALES)  # a * 2 leaves the ellipse domain
    with pytest.raises(c3x.C3XError, match="scale 0"):
        _run(c3x, dev, cat, 0, [1e-7, 1.0])  # b * 1e-7 leaves it too
