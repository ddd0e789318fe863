"""GPU parity at the full sizes the benchmark reports, in its launch
configuration (one c3x_build_index + c3x_match, or one batch plan and its
graph replays), both precisions:

* 200M x 200M full sky with galactic-plane clustering, r = 1.5": 2,000 A
  rows (half within 5 deg of the galactic plane, half beyond 30 deg)
  checked one by one against the oracle over every B row that could match
  them; the full result's canonical order, radius bound and size;
* 100k galactic ellipses against 50M in-band sources: 4,000 sampled rows,
  the same way;
* the 4,096-job batch: every job against the oracle run on that job.

The oracle's B set for sampled rows is every B row whose Dec lies within
the reach of a sampled row's Dec (a superset of the candidates: two points
closer than the reach differ in Dec by less than it), found with Dec bins
one reach wide.
"""
import numpy as np
import pytest

import synth
from test_gpu_parity import SEP_TOL, _t, gpu_match
from test_gpu_batch import check_batch

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


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


def near_dec_subset(dec_rows, decB, reach_arcsec):
    """Sorted indices of the B rows within reach_arcsec in Dec of some row."""
    w = reach_arcsec / 3600.0
    nb = int(np.ceil(180.0 / w)) + 2
    mark = np.zeros(nb + 2, dtype=bool)
    br = np.floor((dec_rows + 90.0) / w).astype(np.int64)
    for o in (-1, 0, 1):
        mark[np.clip(br + o, 0, nb + 1)] = True
    bb = np.clip(np.floor((decB + 90.0) / w).astype(np.int64), 0, nb + 1)
    return np.nonzero(mark[bb])[0]


def check_sampled(g, rows, sub, o, nA):
    """GPU pairs of the sampled rows against the oracle run on those rows
    (indices rows[k]) and B rows sub[j]."""
    mark = np.zeros(nA, dtype=bool)
    mark[rows] = True
    sel = mark[g["ia"]]
    remap = np.searchsorted(rows, g["ia"][sel])
    assert np.array_equal(remap, o.ia)
    assert np.array_equal(g["ib"][sel], sub[o.ib])
    if sel.any():
        assert np.abs(g["sep"][sel] - o.sep).max() <= SEP_TOL
    if "best" in g:
        ob = np.where(o.best_idx >= 0, sub[np.maximum(o.best_idx, 0)], -1)
        assert np.array_equal(g["best"][rows], ob)
        m = o.best_idx >= 0
        assert np.abs(g["best_sep"][rows][m] - o.best_sep[m]).max() <= SEP_TOL


def check_canonical(g, reach_arcsec):
    key = g["ia"].astype(np.int64) * (1 << 31) + g["ib"]
    assert np.all(np.diff(key) > 0)
    assert g["sep"].max() <= reach_arcsec + 1e-9


# ---------------------------------------------------------------------------- 200M x 200M

def _sin_b(ra, dec):
    """sin of galactic latitude: the unit vector against the galactic pole's."""
    a0, d0 = np.radians(192.85948), np.radians(27.12825)
    r, d = np.radians(ra), np.radians(dec)
    return (np.cos(d) * np.cos(d0) * np.cos(r - a0) + np.sin(d) * np.sin(d0))


@pytest.fixture(scope="module")
def cfg5():
    import oracle
    import time
    t = time.time()
    cat = synth.cfg5_scale(scale=1.0)
    print(f"[gpu] cfg5 generated in {time.time() - t:.0f}s", flush=True)
    rng = np.random.default_rng(21)
    pick = rng.choice(cat.nA, 400_000, replace=False)
    sb = np.abs(_sin_b(cat.raA[pick], cat.decA[pick]))
    plane = pick[sb < np.sin(np.radians(5.0))][:1000]
    high = pick[sb > np.sin(np.radians(30.0))][:1000]
    rows = np.unique(np.concatenate([plane, high]))
    assert rows.shape[0] == 2000
    sub = near_dec_subset(cat.decA[rows], cat.decB, cat.radius_arcsec)
    o = oracle.match(cat.raA[rows], cat.decA[rows], cat.raB[sub], cat.decB[sub],
                     radius_arcsec=cat.radius_arcsec)
    print(f"[gpu] cfg5 oracle on {rows.shape[0]} rows x {sub.shape[0]} B done", flush=True)
    return cat, rows, sub, o


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision", [1, 0])
def test_cfg5_full_size_sampled(c3x, dev, cfg5, precision):
    cat, rows, sub, o = cfg5
    g = gpu_match(c3x, dev, cat, precision)
    check_sampled(g, rows, sub, o, cat.nA)
    assert len(o.ia) > 800  # about half the rows have their copy within 1.5"
    check_canonical(g, cat.radius_arcsec)
    assert 0.9e8 < len(g["ia"]) < 1.15e8


# ---------------------------------------------------------------------------- 100k x 50M ellipses

@pytest.fixture(scope="module")
def cfg3():
    import oracle
    cat = synth.cfg3_galactic_ellipses(scale=1.0)
    rows = np.sort(np.random.default_rng(22).choice(cat.nA, 4000, replace=False))
    sub = near_dec_subset(cat.decA[rows], cat.decB, 60.0)
    o = oracle.match(cat.raA[rows], cat.decA[rows], cat.raB[sub], cat.decB[sub], shape=1,
                     a=cat.a_arcsec[rows], b=cat.b_arcsec[rows], pa=cat.pa_deg[rows],
                     pa_zero_deg=cat.pa_zero_deg, pa_sense=cat.pa_sense)
    return cat, rows, sub, o


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precision", [1, 0])
def test_cfg3_full_size_sampled(c3x, dev, cfg3, precision):
    cat, rows, sub, o = cfg3
    g = gpu_match(c3x, dev, cat, precision, mode=1)
    g.pop("best")
    check_sampled(g, rows, sub, o, cat.nA)
    assert len(o.ia) > 100_000
    check_canonical(g, 60.0)
    assert 3.5e6 < len(g["ia"]) < 5e6


# ---------------------------------------------------------------------------- 4,096 jobs

@pytest.fixture(scope="module")
def cfg4():
    import oracle
    cat = synth.cfg4_jobs(scale=1.0)
    jobs = [tuple(int(v) for v in r[:4]) + (float(r[4]),) for r in cat.jobs]
    ors = [oracle.match(cat.raA[ao:ao + na], cat.decA[ao:ao + na], cat.raB[bo:bo + nb],
                        cat.decB[bo:bo + nb], radius_arcsec=r) for ao, na, bo, nb, r in jobs]
    return cat, jobs, ors


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision", [1, 0])
def test_cfg4_every_job_full_size(c3x, dev, cfg4, precision):
    cat, jobs, ors = cfg4
    assert len(jobs) == 4096 and cat.nB > 1e8
    print(f"[gpu] cfg4 batch precision={precision}", flush=True)
    b = c3x.Batch(jobs, _t(cat.raA, dev), _t(cat.decA, dev), _t(cat.raB, dev),
                  _t(cat.decB, dev), precision=precision)
    check_batch(b.result(), b.pair_offsets(), jobs, ors)
    b.run()  # a graph replay, as the benchmark times it
    check_batch(b.result(), b.pair_offsets(), jobs, ors)
    b.free()
