"""GPU parity on the paths and configurations the other GPU tests leave
out, each against the CPU oracle:

* the one-sweep radix schedule on small inputs, and its bounded look-back
  forced to give up (a host setting makes every tile but the first give
  up at once, so every kernel still ends normally): the index build, the
  match (A order and long-segment sorts) and the batch must notice, redo
  their work with the table schedule and return the oracle's answer;
* ellipses around the poles (sources exactly on both poles) and across
  RA = 0/360 (paper Section 2.1, the area centred on the A source);
* the batch's host binary128 decisions and best-match tie ranking, driven
  by near-boundary rows and mirror-image exact ties;
* the forced decision paths (host settings; the answer must not change):
  every candidate within twice the area listed for the FP64 recheck, and
  every band candidate and every best match of a row with two or more
  matches decided in binary128 on the host;
* c3x_result_copy into host and device buffers;
* allocation failure at every allocation of a call: C3X_ENOMEM, no
  result, nothing left allocated.
"""
import ctypes

import numpy as np
import pytest

import synth
from test_gpu_parity import SEP_TOL, _t, assert_parity, gpu_match, oracle_match
from test_gpu_batch import check_batch, small_batch

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


@pytest.fixture(scope="module")
def cfg2_small():
    return synth.cfg2_fullsky(scale=0.002)


@pytest.fixture(scope="module")
def cfg2_small_oracle(cfg2_small):
    return oracle_match(cfg2_small)


def _match_with_stats(c3x, dev, cat, precision):
    print(f"[gpu] {cat.name} precision={precision}", flush=True)
    ix = c3x.build_index(_t(cat.raB, dev), _t(cat.decB, dev), frame=cat.frame,
                         reach_hint_arcsec=cat.reach_arcsec(), precision=precision)
    kw = dict(shape=0, radius_arcsec=cat.radius_arcsec)
    if cat.shape == 1:
        kw = dict(shape=1, a=_t(cat.a_arcsec, dev), b=_t(cat.b_arcsec, dev),
                  pa=_t(cat.pa_deg, dev), pa_zero_deg=cat.pa_zero_deg, pa_sense=cat.pa_sense)
    r = c3x.match(ix, _t(cat.raA, dev), _t(cat.decA, dev), frame=cat.frame, **kw)
    ist = ix.stats()
    ix.free()
    g = dict(ia=r.idxA.cpu().numpy(), ib=r.idxB.cpu().numpy(), sep=r.sep.cpu().numpy(),
             best=r.best_idx.cpu().numpy(), best_sep=r.best_sep.cpu().numpy(), stats=r.stats)
    return g, ist


# ---------------------------------------------------------------------------- one-sweep sort

@pytest.mark.parametrize("precision", [0, 1])
def test_one_sweep_schedule_small(c3x, dev, cfg2_small, cfg2_small_oracle, precision, monkeypatch):
    """Every sort takes the one-sweep schedule (from one tile up)."""
    monkeypatch.setenv("C3X_DEBUG_ONESWEEP_TILES", "1")
    g, ist = _match_with_stats(c3x, dev, cfg2_small, precision)
    assert_parity(g, cfg2_small_oracle)
    assert ist["n_sort_retries"] == 0 and g["stats"]["n_sort_retries"] == 0


@pytest.mark.parametrize("items", ["16", "24"])
def test_one_sweep_other_tiles(c3x, dev, cfg2_small, cfg2_small_oracle, items, monkeypatch):
    """One-sweep passes over tiles of 256 x 16 and 256 x 24 elements (the
    default is 256 x 32)."""
    monkeypatch.setenv("C3X_DEBUG_ONESWEEP_TILES", "1")
    monkeypatch.setenv("C3X_ONESWEEP_ITEMS", items)
    g, ist = _match_with_stats(c3x, dev, cfg2_small, 1)
    assert_parity(g, cfg2_small_oracle)
    assert ist["n_sort_retries"] == 0 and g["stats"]["n_sort_retries"] == 0


@pytest.mark.parametrize("precision", [0, 1])
def test_one_sweep_give_up_is_redone(c3x, dev, cfg2_small, cfg2_small_oracle, precision,
                                     monkeypatch):
    """Spin limit 0: every look-back but the first tile's gives up at once.
    The index build and the match see it and redo their work with the
    table schedule; the answer is the oracle's."""
    monkeypatch.setenv("C3X_DEBUG_ONESWEEP_TILES", "1")
    monkeypatch.setenv("C3X_DEBUG_SORT_SPIN", "0")
    assert cfg2_small.nA > 3 * 4096 and cfg2_small.nB > 3 * 4096  # several tiles
    g, ist = _match_with_stats(c3x, dev, cfg2_small, precision)
    assert_parity(g, cfg2_small_oracle)
    assert ist["n_sort_retries"] == 1
    assert g["stats"]["n_sort_retries"] == 1


def test_one_sweep_give_up_in_long_segments(c3x, dev, monkeypatch):
    """Rows with tens of thousands of matches are ordered by two radix sorts
    of their entries; a give-up there redoes the call too."""
    g = np.random.default_rng(11)
    rb, db = synth.cap_uniform(g, 120_000, 40.0, -30.0, 0.3)
    ra, da = synth.cap_uniform(g, 8, 40.0, -30.0, 0.05)
    cat = synth.Catalogues("long_segments_giveup", ra, da, rb, db, radius_arcsec=400.0)
    o = oracle_match(cat)
    assert np.bincount(o.ia).max() > 2048
    monkeypatch.setenv("C3X_DEBUG_ONESWEEP_TILES", "1")
    monkeypatch.setenv("C3X_DEBUG_SORT_SPIN", "0")
    for precision in (0, 1):
        gm, _ = _match_with_stats(c3x, dev, cat, precision)
        assert_parity(gm, o)
        assert gm["stats"]["n_sort_retries"] == 1


def test_batch_give_up_is_redone(c3x, dev, monkeypatch):
    import oracle
    raA, decA, raB, decB, jobs = small_batch(seed=9)
    ors = [oracle.match(raA[ao:ao + na], decA[ao:ao + na], raB[bo:bo + nb], decB[bo:bo + nb],
                        radius_arcsec=r) for ao, na, bo, nb, r in jobs]
    monkeypatch.setenv("C3X_DEBUG_ONESWEEP_TILES", "1")
    monkeypatch.setenv("C3X_DEBUG_SORT_SPIN", "0")
    assert sum(j[3] for j in jobs) > 3 * 4096
    print("[gpu] batch with forced sort give-up", flush=True)
    b = c3x.Batch(jobs, _t(raA, dev), _t(decA, dev), _t(raB, dev), _t(decB, dev), precision=1)
    check_batch(b.result(), b.pair_offsets(), jobs, ors)
    assert b.stats()["n_sort_retries"] == 1
    b.run()  # the replayed graph was captured with the table schedule
    check_batch(b.result(), b.pair_offsets(), jobs, ors)
    b.free()


# ---------------------------------------------------------------------------- polar ellipses

def _polar_ellipses():
    from test_oracle_pins import _near_boundary_catalogue
    raA, decA, raB, decB, a, b, pa = _near_boundary_catalogue(41, 120, 1500, 1, lat=(88.0, 90.0))
    r2A, d2A, r2B, d2B, a2, b2, pa2 = _near_boundary_catalogue(42, 60, 700, 1,
                                                               lat=(-90.0, -88.0))
    g = np.random.default_rng(43)
    # sources exactly on each pole, and ellipses across RA = 0/360
    xa = np.array([0.0, 123.4, 0.0, 271.0, 359.99999, 0.00001, 359.9996, 0.0])
    xd = np.array([90.0, 90.0, -90.0, -90.0, 12.0, -40.0, 0.0, 65.0])
    xA = np.array([60.0, 30.0, 45.0, 20.0, 50.0, 40.0, 25.0, 58.0])
    xB = xA * np.array([0.3, 1.0, 0.5, 0.9, 0.4, 0.7, 0.35, 0.6])
    xpa = np.array([0.0, 77.0, 135.0, 10.0, 90.0, 45.0, 170.0, 5.0])
    rb, db = [], []
    for k in range(xa.shape[0]):
        n = 150
        rr, dd = synth.destination(np.full(n, xa[k]), np.full(n, xd[k]),
                                   g.uniform(0, 360, n), xA[k] * g.uniform(0.2, 1.3, n) / 3600)
        rb.append(rr)
        db.append(dd)
    cat = synth.Catalogues("polar_ellipses", np.concatenate([raA, r2A, xa]),
                           np.concatenate([decA, d2A, xd]),
                           np.concatenate([raB, r2B] + rb), np.concatenate([decB, d2B] + db),
                           shape=1, pa_zero_deg=7.0, pa_sense=-1)
    cat.a_arcsec = np.concatenate([a, a2, xA])
    cat.b_arcsec = np.concatenate([b, b2, xB])
    cat.pa_deg = np.concatenate([pa, pa2, xpa])
    return cat


@pytest.mark.parametrize("precision", [0, 1])
def test_polar_and_wrap_ellipses(c3x, dev, precision):
    cat = _polar_ellipses()
    o = oracle_match(cat)
    n0 = cat.nA - 8
    pole_rows = np.isin(o.ia, np.arange(n0, n0 + 4))
    assert pole_rows.sum() > 100 and len(o.ia) > 1000
    g = gpu_match(c3x, dev, cat, precision)
    assert_parity(g, o)


# ---------------------------------------------------------------------------- batch fallbacks

def _batch_fallback_data():
    """One job per adversarial centre (B at r(1 +- 2^-45), r(1 +- 2^-30), r,
    r/2, 2r: the FP64 recheck cannot decide the first two), plus jobs whose
    A sources have pairs of B at exactly equal distances (mirror images
    about the source on its meridian and on the equator)."""
    c = synth.adversarial_circle(radius_arcsec=1.0, n_centres=48)
    nc = c.nA
    raA, decA, raB, decB, jobs = [], [], [], [], []
    na = nb = 0
    per = c.nB // nc
    for k in range(nc):
        sel = np.arange(k, c.nB, nc)  # the placements around centre k
        assert sel.shape[0] == per
        raA.append(c.raA[k:k + 1])
        decA.append(c.decA[k:k + 1])
        raB.append(c.raB[sel])
        decB.append(c.decB[sel])
        jobs.append((na, 1, nb, per, 1.0))
        na += 1
        nb += per
    # exact ties: d = 2^-14 deg (dyadic, so ra +- d and +-d are exact)
    d = 2.0 ** -14
    for ra0 in (100.0, 17.0, 250.0):
        ra_t = np.array([ra0, ra0 + 0.25])
        de_t = np.array([0.0, 0.0])
        rb_t = np.array([ra0 + d, ra0 - d, ra0, ra0, ra0 + 0.25 + 2 * d, ra0 + 0.25 - 2 * d])
        db_t = np.array([0.0, 0.0, d, -d, 0.0, 0.0])
        raA.append(ra_t)
        decA.append(de_t)
        raB.append(rb_t)
        decB.append(db_t)
        jobs.append((na, 2, nb, 6, 3.0))
        na += 2
        nb += 6
    return (np.concatenate(raA), np.concatenate(decA), np.concatenate(raB),
            np.concatenate(decB), jobs)


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_binary128_and_tie_paths(c3x, dev, precision):
    import oracle
    raA, decA, raB, decB, jobs = _batch_fallback_data()
    ors = [oracle.match(raA[ao:ao + na], decA[ao:ao + na], raB[bo:bo + nb], decB[bo:bo + nb],
                        radius_arcsec=r) for ao, na, bo, nb, r in jobs]
    assert sum(o.n_ambiguous for o in ors) > 0 and sum(o.n_best_ties for o in ors) > 0
    print(f"[gpu] batch fallback paths precision={precision}", flush=True)
    b = c3x.Batch(jobs, _t(raA, dev), _t(decA, dev), _t(raB, dev), _t(decB, dev),
                  precision=precision)
    st = b.stats()
    assert st["n_ambiguous"] > 0, st
    assert st["n_best_ties"] > 0, st
    check_batch(b.result(), b.pair_offsets(), jobs, ors)
    for _ in range(2):  # the host node runs on every replay
        b.run()
        check_batch(b.result(), b.pair_offsets(), jobs, ors)
    # the exact ties went to the lower B row
    best = b.result().best_idx.cpu().numpy()
    a0 = sum(j[1] for j in jobs[:-3])
    assert best[a0:].tolist() == [0, 4, 0, 4, 0, 4]
    b.free()


# ---------------------------------------------------------------------------- result copy

# ---------------------------------------------------------------------------- forced decisions

_FORCED = {}


def _forced_case(shape):
    """Circles: the 10k-source patch; ellipses and rectangles: a small draw
    of the galactic-plane ellipse catalogue (the same axes taken as half
    sides); each with the oracle's answer, computed once."""
    if shape not in _FORCED:
        if shape == 0:
            cat = synth.cfg1_patch()
        else:
            cat = synth.cfg3_galactic_ellipses(scale=0.001)
            cat.shape = shape
        _FORCED[shape] = (cat, oracle_match(cat))
    return _FORCED[shape]


@pytest.mark.parametrize("shape", [0, 1, 2])
@pytest.mark.parametrize("knobs", ["C3X_DEBUG_FORCE_BAND", "C3X_DEBUG_FORCE_AMBIG",
                                   "C3X_DEBUG_FORCE_BAND,C3X_DEBUG_FORCE_AMBIG"])
def test_forced_decision_paths(c3x, dev, shape, knobs, monkeypatch):
    """FORCE_BAND: the filter decides nothing inside, so every match comes
    through the band list, the FP64 recheck and the re-ranking of rows with a
    band match. FORCE_AMBIG: the recheck and the FP64 ranking let nothing
    stand, so every band candidate and every best match among two or more
    goes to binary128 on the host. Both precisions, the oracle's answer."""
    cat, o = _forced_case(shape)
    assert len(o.ia) > 1000
    for k in knobs.split(","):
        monkeypatch.setenv(k, "1")
    multi = int((np.bincount(o.ia, minlength=len(cat.raA)) >= 2).sum())
    assert multi > 0
    for precision in (0, 1):
        print(f"[gpu] forced {knobs} shape={shape} precision={precision}", flush=True)
        g = gpu_match(c3x, dev, cat, precision)
        assert_parity(g, o)
        st = g["stats"]
        if "BAND" in knobs:
            assert st["n_band"] >= len(o.ia)
        if "AMBIG" in knobs:  # (alone, the band may be empty: then only ties)
            assert st["n_ambiguous"] == st["n_band"]
            assert st["n_best_ties"] >= multi


@pytest.mark.parametrize("where", ["cpu", "cuda"])
def test_result_copy(c3x, dev, cfg2_small, cfg2_small_oracle, where):
    import torch
    cat = cfg2_small
    ix = c3x.build_index(_t(cat.raB, dev), _t(cat.decB, dev), reach_hint_arcsec=cat.radius_arcsec,
                         precision=1)
    r = c3x.match(ix, _t(cat.raA, dev), _t(cat.decA, dev), radius_arcsec=cat.radius_arcsec)
    ix.free()
    d = torch.device(where) if where == "cpu" else dev
    P, n = r.n_pairs, cat.nA
    out = dict(idxA=torch.full((P,), -7, dtype=torch.int32, device=d),
               idxB=torch.full((P,), -7, dtype=torch.int32, device=d),
               sep=torch.full((P,), -7.0, dtype=torch.float64, device=d),
               best_idx=torch.full((n,), -7, dtype=torch.int32, device=d),
               best_sep=torch.full((n,), -7.0, dtype=torch.float64, device=d))
    if where == "cpu":
        out = {k: v.pin_memory() if k == "sep" else v for k, v in out.items()}
    c3x.result_copy(r, **out)
    g = {k: v.cpu().numpy() for k, v in out.items()}
    g = dict(ia=g["idxA"], ib=g["idxB"], sep=g["sep"], best=g["best_idx"], best_sep=g["best_sep"])
    assert_parity(g, cfg2_small_oracle)
    # any subset; NULL for the rest
    only = torch.zeros(n, dtype=torch.int32, device=d)
    c3x.result_copy(r, best_idx=only)
    assert np.array_equal(only.cpu().numpy(), cfg2_small_oracle.best_idx)


# ---------------------------------------------------------------------------- allocation failure

def test_allocation_failure_is_clean(c3x, dev, cfg2_small):
    """The k-th device allocation of a call fails, for every k: the call
    either succeeds (fewer allocations than k) or returns C3X_ENOMEM with
    *out NULL, and the library then holds no more device blocks than
    before."""
    import torch
    L = c3x.lib()
    L.c3x_debug_live_blocks.restype = ctypes.c_int
    L.c3x_debug_fail_alloc.argtypes = [ctypes.c_int]
    L.c3x_debug_fail_alloc.restype = None
    cat = cfg2_small
    raB, decB, raA, decA = (_t(x, dev) for x in (cat.raB, cat.decB, cat.raA, cat.decA))
    Opts, Area = c3x._binding.Opts, c3x._binding.Area
    o = Opts(precision=1, cell_arcsec=0.0, tile=0, stream=None)
    ar = Area(shape=0, radius_arcsec=cat.radius_arcsec, pa_zero_deg=0.0, pa_sense=1)

    def build(k):
        ix = ctypes.c_void_p(0x1234)
        L.c3x_debug_fail_alloc(k)
        st = L.c3x_build_index(raB.data_ptr(), decB.data_ptr(), cat.nB, 0, 2.0,
                               ctypes.byref(o), ctypes.byref(ix))
        L.c3x_debug_fail_alloc(0)
        return st, ix

    def match(ix, k):
        out = ctypes.c_void_p(0x1234)
        L.c3x_debug_fail_alloc(k)
        st = L.c3x_match(ix, raA.data_ptr(), decA.data_ptr(), cat.nA, 0, ctypes.byref(ar), 3,
                         ctypes.byref(o), ctypes.byref(out))
        L.c3x_debug_fail_alloc(0)
        return st, out

    st, ix = build(0)  # warm-up: zone tables and caches in place
    assert st == 0
    st, out = match(ix, 0)
    assert st == 0
    L.c3x_result_free(out)
    L.c3x_index_free(ix)
    torch.cuda.synchronize()
    base = L.c3x_debug_live_blocks()
    fails = {"index": 0, "match": 0}
    for k in range(1, 80):
        print(f"[gpu] allocation {k} fails", flush=True)
        st, ix = build(k)
        if st == 0:
            L.c3x_index_free(ix)
        else:
            assert st == 3, (k, st, L.c3x_last_error())
            assert ix.value is None
            fails["index"] += 1
        assert L.c3x_debug_live_blocks() == base, ("index", k)
        st, ix = build(0)
        assert st == 0
        st, out = match(ix, k)
        if st == 0:
            L.c3x_result_free(out)
        else:
            assert st == 3, (k, st, L.c3x_last_error())
            assert out.value is None
            fails["match"] += 1
        L.c3x_index_free(ix)
        torch.cuda.synchronize()
        assert L.c3x_debug_live_blocks() == base, ("match", k)
    assert fails["match"] >= 20 and fails["index"] >= 5, fails
