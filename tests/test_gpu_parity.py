"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Pair sets and best-match indices must be identical; separations agree to
1e-6 arcsec. Covered: the 10k x 10k patch in full, both precisions; the
closed-form fixtures; adversarial near-boundary rows; scaled-down full-sky
(RA wrap, polar cap) and galactic-ellipse workloads; several cell sizes;
BEST-only output; radius 0 and duplicates; empty inputs; error paths;
sampled rows of the full 10M x 10M full-sky workload; and sampled rows of a
34M x 34M full-sky draw (sorted by the one-sweep passes).
"""
import os
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

SEP_TOL = 1e-6  # arcsec


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


def gpu_match(c3x, dev, cat, precision, mode=3, cell_arcsec=0.0, reach=None):
    print(f"[gpu] {cat.name} precision={precision} mode={mode} cell={cell_arcsec}", flush=True)
    ix = c3x.build_index(_t(cat.raB, dev), _t(cat.decB, dev), frame=cat.frame,
                         reach_hint_arcsec=cat.reach_arcsec() if reach is None else reach,
                         precision=precision, cell_arcsec=cell_arcsec)
    kw = {}
    if cat.shape in (1, 2):
        kw = dict(shape=cat.shape, a=_t(cat.a_arcsec, dev), b=_t(cat.b_arcsec, dev),
                  pa=_t(cat.pa_deg, dev), pa_zero_deg=cat.pa_zero_deg, pa_sense=cat.pa_sense)
    else:
        kw = dict(shape=0, radius_arcsec=cat.radius_arcsec)
    r = c3x.match(ix, _t(cat.raA, dev), _t(cat.decA, dev), frame=cat.frame, mode=mode, **kw)
    ix.free()
    return dict(ia=r.idxA.cpu().numpy(), ib=r.idxB.cpu().numpy(), sep=r.sep.cpu().numpy(),
                best=r.best_idx.cpu().numpy(), best_sep=r.best_sep.cpu().numpy(), stats=r.stats)


def oracle_match(cat, **kw):
    import oracle
    a = dict(shape=cat.shape, radius_arcsec=cat.radius_arcsec)
    if cat.shape in (1, 2):
        a.update(a=cat.a_arcsec, b=cat.b_arcsec, pa=cat.pa_deg, pa_zero_deg=cat.pa_zero_deg,
                 pa_sense=cat.pa_sense)
    a.update(kw)
    return oracle.match(cat.raA, cat.decA, cat.raB, cat.decB, **a)


def assert_parity(g, o, best=True):
    assert g["ia"].shape == o.ia.shape, (g["ia"].shape, o.ia.shape)
    assert np.array_equal(g["ia"], o.ia)
    assert np.array_equal(g["ib"], o.ib)
    d = np.abs(g["sep"] - o.sep)
    assert d.size == 0 or d.max() <= SEP_TOL, d.max()
    if best:
        assert np.array_equal(g["best"], o.best_idx)
        m = o.best_idx >= 0
        assert np.all(np.isnan(g["best_sep"][~m]))
        if m.any():
            assert np.abs(g["best_sep"][m] - o.best_sep[m]).max() <= SEP_TOL


@pytest.fixture(scope="module")
def cfg1():
    return synth.cfg1_patch()


@pytest.fixture(scope="module")
def cfg1_oracle(cfg1):
    return oracle_match(cfg1)


@pytest.mark.parametrize("precision", [0, 1])
def test_cfg1_patch_full(c3x, dev, cfg1, cfg1_oracle, precision):
    g = gpu_match(c3x, dev, cfg1, precision)
    assert_parity(g, cfg1_oracle)
    assert 6950 <= len(g["ia"]) <= 7060
    assert g["stats"]["n_tests"] > 0


@pytest.mark.parametrize("precision", [0, 1])
def test_closed_forms(c3x, dev, precision):
    from test_oracle_pins import CLOSED
    groups = {}
    for r in CLOSED:
        groups.setdefault((r["shape"], r["r"], r["pz"], r["sense"]), []).append(r)
    for (shape, rad, pz, sense), rs in groups.items():
        cat = synth.Catalogues(
            "closed", np.array([r["raA"] for r in rs]), np.array([r["decA"] for r in rs]),
            np.array([r["raB"] for r in rs]), np.array([r["decB"] for r in rs]), shape=shape,
            radius_arcsec=rad, pa_zero_deg=pz, pa_sense=sense)
        if shape == 1:
            cat.a_arcsec = np.array([r["a"] for r in rs])
            cat.b_arcsec = np.array([r["b"] for r in rs])
            cat.pa_deg = np.array([r["pa"] for r in rs])
        g = gpu_match(c3x, dev, cat, precision)
        diag = set(int(i) for i, j in zip(g["ia"], g["ib"]) if i == j)
        want = set(k for k, r in enumerate(rs) if r["inside"])
        assert diag == want, (shape, rad, pz, sense)
        assert_parity(g, oracle_match(cat))


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("radius", [1.0, 2.0, 0.25])
def test_adversarial(c3x, dev, precision, radius):
    cat = synth.adversarial_circle(radius_arcsec=radius, n_centres=64)
    o = oracle_match(cat)
    g = gpu_match(c3x, dev, cat, precision)
    assert_parity(g, o)
    assert g["stats"]["n_band"] > 0


@pytest.fixture(scope="module")
def cfg2_small():
    return synth.cfg2_fullsky(scale=0.002)


@pytest.fixture(scope="module")
def cfg2_small_oracle(cfg2_small):
    return oracle_match(cfg2_small)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("cell", [0.0, 2.0, 37.0, 400.0])
def test_cfg2_fullsky_small(c3x, dev, cfg2_small, cfg2_small_oracle, precision, cell):
    g = gpu_match(c3x, dev, cfg2_small, precision, cell_arcsec=cell)
    assert_parity(g, cfg2_small_oracle)


def test_cfg2_large_radius_crosses_poles_and_wrap(c3x, dev):
    cat = synth.cfg2_fullsky(scale=0.0005)
    cat.radius_arcsec = 900.0
    o = oracle_match(cat)
    for precision in (0, 1):
        g = gpu_match(c3x, dev, cat, precision)
        assert_parity(g, o)


@pytest.mark.parametrize("radius_deg", [10.0, 88.0, 90.0])
@pytest.mark.parametrize("precision", [0, 1])
def test_huge_radii(c3x, dev, radius_deg, precision):
    """Radii up to the 90 deg limit (Section 2.1's circle): separations above
    about 5.7 deg are decoded from the chord by the arcsine, above about
    87 deg from both rows' coordinates; both are rare in the hot workloads."""
    rng = np.random.default_rng(synth.SEED_BASE + 777)
    raA, decA = synth.sphere_uniform(rng, 400)
    raB, decB = synth.sphere_uniform(rng, 500)
    cat = synth.Catalogues(f"huge_radius_{radius_deg}", raA, decA, raB, decB,
                           radius_arcsec=radius_deg * 3600.0)
    o = oracle_match(cat)
    assert len(o.ia) > 1000 and np.max(o.sep) > 5.8 * 3600.0
    if radius_deg > 87.5:
        assert np.max(o.sep) > 87.2 * 3600.0
    g = gpu_match(c3x, dev, cat, precision)
    assert_parity(g, o)


@pytest.fixture(scope="module")
def cfg3_small():
    return synth.cfg3_galactic_ellipses(scale=0.003)


@pytest.mark.parametrize("precision", [0, 1])
def test_cfg3_ellipses_small(c3x, dev, cfg3_small, precision):
    o = oracle_match(cfg3_small)
    assert len(o.ia) > 1000
    g = gpu_match(c3x, dev, cfg3_small, precision)
    assert_parity(g, o)


@pytest.mark.parametrize("precision", [0, 1])
def test_ellipse_pa_conventions(c3x, dev, precision):
    cat = synth.cfg3_galactic_ellipses(scale=0.001)
    for pz, sense in ((0.0, 1), (90.0, -1), (-33.0, 1)):
        cat.pa_zero_deg, cat.pa_sense = pz, sense
        assert_parity(gpu_match(c3x, dev, cat, precision), oracle_match(cat))


@pytest.mark.parametrize("precision", [0, 1])
def test_best_only_mode(c3x, dev, cfg1, cfg1_oracle, precision):
    g = gpu_match(c3x, dev, cfg1, precision, mode=2)
    o = cfg1_oracle
    m = o.best_idx >= 0
    assert np.array_equal(g["ia"], np.nonzero(m)[0].astype(np.int32))
    assert np.array_equal(g["ib"], o.best_idx[m])
    assert np.array_equal(g["best"], o.best_idx)


@pytest.mark.parametrize("precision", [0, 1])
def test_zero_radius_and_duplicates(c3x, dev, precision):
    raA = np.array([10.0, 0.0, 0.0, 359.5, 200.0])
    decA = np.array([20.0, 90.0, -90.0, 0.0, -45.0])
    raB = np.array([10.0, 10.0, 123.0, 0.0, 359.5, 359.5, 200.0, 200.0])
    decB = np.array([20.0, 20.0, 90.0, -90.0, 0.0, 1e-300, -45.0, -45.0])
    for r in (0.0, 1.0):
        cat = synth.Catalogues("dups", raA, decA, raB, decB, radius_arcsec=r)
        g = gpu_match(c3x, dev, cat, precision, reach=1.0)
        o = oracle_match(cat)
        assert_parity(g, o)
    assert g["best"][4] == 6   # exact tie between rows 6 and 7 -> lower index


@pytest.mark.parametrize("precision", [0, 1])
def test_empty_inputs(c3x, dev, precision):
    e = np.zeros(0)
    one = np.array([10.0])
    for ra_a, ra_b in ((e, one), (one, e), (e, e)):
        cat = synth.Catalogues("empty", ra_a, ra_a * 0, ra_b, ra_b * 0)
        g = gpu_match(c3x, dev, cat, precision, reach=1.0)
        assert len(g["ia"]) == 0
        assert g["best"].shape == ra_a.shape


def test_errors(c3x, dev):
    bad = _t([10.0, 400.0, 5.0], dev)
    ok = _t([0.0, 0.0, 0.0], dev)
    with pytest.raises(c3x.C3XError, match="row 1"):
        c3x.build_index(bad, ok)
    ix = c3x.build_index(ok, ok, frame=c3x.GALACTIC)
    with pytest.raises(c3x.C3XError, match="row 1"):  # checked before the frame conversion
        c3x.match(ix, bad, ok, frame=c3x.EQUATORIAL)
    with pytest.raises(c3x.C3XError, match="row 2"):
        c3x.match(ix, _t([1.0, 2.0, 3.0], dev), _t([0.0, 0.0, 91.0], dev), frame=c3x.GALACTIC)
    with pytest.raises(c3x.C3XError, match="radius"):
        c3x.match(ix, ok, ok, frame=c3x.GALACTIC, radius_arcsec=-1.0)
    a = _t([10.0, 10.0, 10.0], dev)
    with pytest.raises(c3x.C3XError, match="row 0"):
        c3x.match(ix, ok, ok, frame=c3x.GALACTIC, shape=c3x.ELLIPSE, a=a, b=_t([20.0] * 3, dev),
                  pa=a)
    ix.free()


def test_rerun_is_byte_identical(c3x, dev, cfg2_small):
    g1 = gpu_match(c3x, dev, cfg2_small, 1)
    g2 = gpu_match(c3x, dev, cfg2_small, 1)
    for k in ("ia", "ib", "sep", "best", "best_sep"):
        assert g1[k].tobytes() == g2[k].tobytes()


@pytest.mark.slow
@pytest.mark.parametrize("precision", [1, 0])
def test_cfg2_full_size_sampled(c3x, dev, precision):
    """The 10M x 10M full-sky workload in the benchmark's configuration;
    2,000 A rows (half of them from the dense caps) are checked one by one
    against the oracle run for those rows over the whole of B."""
    import oracle
    import torch
    cat = synth.cfg2_fullsky(scale=1.0)
    g = gpu_match(c3x, dev, cat, precision)
    rng = np.random.default_rng(5)
    dense = np.nonzero(cat.decA > 88.0)[0]
    near0 = np.nonzero((cat.decA > 9.0) & (cat.decA < 11.0) & ((cat.raA < 1.0) | (cat.raA > 359.0)))[0]
    rows = np.unique(np.concatenate([rng.choice(cat.nA, 1000, replace=False),
                                     rng.choice(dense, 500, replace=False),
                                     rng.choice(near0, 500, replace=False)]))
    o = oracle.match(cat.raA[rows], cat.decA[rows], cat.raB, cat.decB,
                     radius_arcsec=cat.radius_arcsec)
    sel = np.isin(g["ia"], rows)
    remap = np.searchsorted(rows, g["ia"][sel])
    assert np.array_equal(remap, o.ia)
    assert np.array_equal(g["ib"][sel], o.ib)
    assert np.abs(g["sep"][sel] - o.sep).max() <= SEP_TOL
    assert np.array_equal(g["best"][rows], o.best_idx)
    # properties at full size: canonical order, seps within the radius
    ia, ib = g["ia"], g["ib"]
    key = ia.astype(np.int64) * (1 << 31) + ib
    assert np.all(np.diff(key) > 0)
    assert g["sep"].max() <= cat.radius_arcsec + 1e-9
    assert 7.0e6 < len(ia) < 8.5e6


@pytest.fixture(scope="module")
def fullsky_34m():
    """A 34M x 34M draw of the full-sky workload (dense caps included): both
    catalogues exceed 32M rows (8,301 tiles of 4,096), so the index and the
    A order are sorted by the one-sweep radix passes (tile prefixes found by
    look-back)."""
    import oracle
    cat = synth.cfg2_fullsky(scale=3.4)
    rng = np.random.default_rng(11)
    dense = np.nonzero(cat.decA > 88.0)[0]
    rows = np.unique(np.concatenate([rng.choice(cat.nA, 1500, replace=False),
                                     rng.choice(dense, 500, replace=False)]))
    o = oracle.match(cat.raA[rows], cat.decA[rows], cat.raB, cat.decB,
                     radius_arcsec=cat.radius_arcsec)
    return cat, rows, o


@pytest.mark.slow
@pytest.mark.parametrize("precision", [1, 0])
def test_one_sweep_sorts_34m_sampled(c3x, dev, fullsky_34m, precision):
    """Sampled rows of a 34M x 34M cross-match against the oracle over the
    whole of B, and the full result's canonical order."""
    cat, rows, o = fullsky_34m
    g = gpu_match(c3x, dev, cat, precision)
    sel = np.isin(g["ia"], rows)
    remap = np.searchsorted(rows, g["ia"][sel])
    assert np.array_equal(remap, o.ia)
    assert np.array_equal(g["ib"][sel], o.ib)
    assert np.abs(g["sep"][sel] - o.sep).max() <= SEP_TOL
    assert np.array_equal(g["best"][rows], o.best_idx)
    key = g["ia"].astype(np.int64) * (1 << 31) + g["ib"]
    assert np.all(np.diff(key) > 0)
    assert g["sep"].max() <= cat.radius_arcsec + 1e-9
    assert len(g["ia"]) > 0.5 * cat.nA


@pytest.mark.parametrize("precision", [0, 1])
def test_long_segments(c3x, dev, precision):
    """Sources with hundreds to tens of thousands of matches each: the
    segment ordering paths beyond the in-kernel rank (LDS bitonic sort and
    the radix-sort fallback) must still give the canonical order."""
    g = np.random.default_rng(11)
    rb, db = synth.cap_uniform(g, 120_000, 40.0, -30.0, 0.3)
    ra1, da1 = synth.cap_uniform(g, 12, 40.0, -30.0, 0.05)      # deep inside: ~40k matches
    ra2, da2 = synth.cap_uniform(g, 40, 40.0, -30.0, 0.3)       # spread: hundreds+
    ra3 = np.array([40.0 + 0.31 / np.cos(np.radians(30.0))])     # just outside the cap
    da3 = np.array([-30.0])
    rb2, db2 = synth.cap_uniform(g, 700, 200.0, 10.0, 0.05)     # a small cluster: ~700 matches
    ra4, da4 = synth.cap_uniform(g, 5, 200.0, 10.0, 0.01)
    cat = synth.Catalogues("long_segments", np.concatenate([ra1, ra2, ra3, ra4]),
                           np.concatenate([da1, da2, da3, da4]), np.concatenate([rb, rb2]),
                           np.concatenate([db, db2]), radius_arcsec=400.0)
    o = oracle_match(cat)
    seg = np.bincount(o.ia, minlength=cat.nA)
    assert seg.max() > 2048 and ((seg > 64) & (seg <= 2048)).any()
    assert_parity(gpu_match(c3x, dev, cat, precision), o)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("slots", ["0", "1", "100000"])
def test_write_pass_fallback(c3x, dev, cfg2_small, cfg2_small_oracle, precision, slots,
                             monkeypatch):
    """Without the table (0), with overflow regions too small for the
    matches beyond a row's table slots (1 slot each), and with ample ones:
    when the single pass cannot keep every match the count stands and the
    write pass puts them in place. The result is the same."""
    monkeypatch.setenv("C3X_DEBUG_OVERFLOW_SLOTS", slots)
    assert_parity(gpu_match(c3x, dev, cfg2_small, precision), cfg2_small_oracle)


@pytest.mark.parametrize("precision", [0, 1])
def test_dense_emission(c3x, dev, precision):
    """Sources with 0 to about a dozen matches each inside one dense patch
    (about 1.5 per source): many rows fill their table slots and spill into
    the overflow list."""
    g = np.random.default_rng(12)
    rb, db = synth.cap_uniform(g, 200_000, 300.0, 45.0, 0.2)
    ra, da = synth.cap_uniform(g, 30_000, 300.0, 45.0, 0.22)
    cat = synth.Catalogues("dense_emission", ra, da, rb, db, radius_arcsec=2.2)
    o = oracle_match(cat)
    seg = np.bincount(o.ia, minlength=cat.nA)
    assert seg.max() >= 8 and 1.5 * cat.nA < len(o.ia) < 2 * cat.nA
    assert_parity(gpu_match(c3x, dev, cat, precision), o)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("wide_min", ["0", "1", "4"])
def test_wavefront_rows(c3x, dev, cfg2_small, cfg2_small_oracle, cfg3_small, precision, wide_min,
                        monkeypatch):
    """Rows counted one lane each (0), every row by a wavefront of its own (1),
    and a split at 4 candidates: the same pairs, best matches, band decisions
    and near-tie re-ranking, in all-matches and best-only modes."""
    monkeypatch.setenv("C3X_WIDE_MIN", wide_min)
    assert_parity(gpu_match(c3x, dev, cfg2_small, precision), cfg2_small_oracle)
    g = gpu_match(c3x, dev, cfg2_small, precision, mode=2)
    m = cfg2_small_oracle.best_idx >= 0
    assert np.array_equal(g["ib"], cfg2_small_oracle.best_idx[m])
    assert np.array_equal(g["best"], cfg2_small_oracle.best_idx)
    assert_parity(gpu_match(c3x, dev, cfg3_small, precision), oracle_match(cfg3_small))
    cat = synth.adversarial_circle(radius_arcsec=1.0, n_centres=64)
    g = gpu_match(c3x, dev, cat, precision)
    assert_parity(g, oracle_match(cat))
    assert g["stats"]["n_band"] > 0
    r = np.random.default_rng(5)
    rb, db = synth.cap_uniform(r, 60_000, 300.0, 45.0, 0.1)
    ra, da = synth.cap_uniform(r, 8_000, 300.0, 45.0, 0.11)
    cat = synth.Catalogues("dense_wave", ra, da, rb, db, radius_arcsec=4.0)
    assert_parity(gpu_match(c3x, dev, cat, precision), oracle_match(cat))


def test_result_views_outlive_the_result_object(c3x, dev, cfg2_small):
    """The output tensors view the library's own arrays: they stay valid
    after the result object is gone and while other calls run."""
    import gc
    import torch
    print("[gpu] result views lifetime", flush=True)
    t = [_t(x, dev) for x in (cfg2_small.raA, cfg2_small.decA, cfg2_small.raB, cfg2_small.decB)]
    ix = c3x.build_index(t[2], t[3], reach_hint_arcsec=cfg2_small.radius_arcsec)
    r = c3x.match(ix, t[0], t[1], radius_arcsec=cfg2_small.radius_arcsec)
    ia, sep = r.idxA, r.sep
    want_ia, want_sep = ia.cpu().numpy().copy(), sep.cpu().numpy().copy()
    del r
    gc.collect()
    for _ in range(3):  # later calls must not reuse the viewed arrays
        r2 = c3x.match(ix, t[0], t[1], radius_arcsec=2 * cfg2_small.radius_arcsec)
        del r2
    torch.cuda.synchronize()
    assert np.array_equal(ia.cpu().numpy(), want_ia)
    assert np.array_equal(sep.cpu().numpy(), want_sep)
    ix.free()
