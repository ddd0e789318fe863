"""GPU parity of the batched form: every job of a batch against the CPU
oracle run on that job alone (pairs, best indices, separations within
1e-6 arcsec), graph replays identical to the plan's run, and the plan's
errors."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

SEP_TOL = 1e-6


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


def small_batch(seed=5):
    """Jobs on 0.5 deg caps: at the RA seam, at both poles, on the equator
    and at random places; sizes from 0 to a few thousand; radii 0.5-10"; a
    zero-radius job with exact duplicates; a job reusing another's rows."""
    g = np.random.default_rng(seed)
    centres = [(0.05, 10.0), (359.95, -5.0), (180.0, 89.8), (45.0, -89.7), (90.0, 0.0)]
    centres += list(zip(*synth.sphere_uniform(g, 19)))
    sizes = [2000, 500, 800, 300, 37, 1, 0, 1500, 60, 900, 120, 2500, 10, 400, 700, 50, 1000,
             250, 3, 600, 90, 1200, 5, 333]
    raA, decA, raB, decB, jobs = [], [], [], [], []
    na_tot = nb_tot = 0
    for k, ((rc, dc), n) in enumerate(zip(centres, sizes)):
        ra, de = synth.cap_uniform(g, n, rc, dc, 0.5)
        nj = n // 2
        par = g.choice(max(n, 1), size=nj, replace=False) if n else np.array([], dtype=int)
        rj, dj = synth.jitter(g, ra[par], de[par], 0.3) if nj else (np.array([]), np.array([]))
        rr, dr = synth.cap_uniform(g, 5 * n + 3, rc, dc, 0.5)
        rb, db = np.concatenate([rj, rr]), np.concatenate([dj, dr])
        r = float(g.uniform(0.5, 10.0))
        if k == 8:  # radius 0 with duplicated positions
            r = 0.0
            rb = np.concatenate([rb, ra[:20]])
            db = np.concatenate([db, de[:20]])
        raA.append(ra)
        decA.append(de)
        raB.append(rb)
        decB.append(db)
        jobs.append((na_tot, len(ra), nb_tot, len(rb), r))
        na_tot += len(ra)
        nb_tot += len(rb)
    jobs.append(jobs[0][:4] + (3.5,))  # same rows as job 0, another radius
    return (np.concatenate(raA), np.concatenate(decA), np.concatenate(raB),
            np.concatenate(decB), jobs)


@pytest.fixture(scope="module")
def batch_data():
    return small_batch()


@pytest.fixture(scope="module")
def batch_oracle(batch_data):
    import oracle
    raA, decA, raB, decB, jobs = batch_data
    out = []
    for ao, na, bo, nb, r in jobs:
        out.append(oracle.match(raA[ao:ao + na], decA[ao:ao + na], raB[bo:bo + nb],
                                decB[bo:bo + nb], radius_arcsec=r))
    return out


def check_batch(res, offs, jobs, oracles):
    ia, ib = res.idxA.cpu().numpy(), res.idxB.cpu().numpy()
    sep, best = res.sep.cpu().numpy(), res.best_idx.cpu().numpy()
    bsep = res.best_sep.cpu().numpy()
    a0 = 0
    for k, ((ao, na, bo, nb, r), o) in enumerate(zip(jobs, oracles)):
        p0, p1 = offs[k], offs[k + 1]
        assert np.array_equal(ia[p0:p1], o.ia), k
        assert np.array_equal(ib[p0:p1], o.ib), k
        if p1 > p0:
            assert np.abs(sep[p0:p1] - o.sep).max() <= SEP_TOL, k
        assert np.array_equal(best[a0:a0 + na], o.best_idx), k
        m = o.best_idx >= 0
        assert np.all(np.isnan(bsep[a0:a0 + na][~m])), k
        if m.any():
            assert np.abs(bsep[a0:a0 + na][m] - o.best_sep[m]).max() <= SEP_TOL, k
        a0 += na
    assert offs[-1] == len(ia)


@pytest.mark.parametrize("precision,queue", [(0, None), (1, None), (0, "1"), (1, "1")])
def test_batch_matches_oracle_per_job(c3x, dev, batch_data, batch_oracle, precision, queue,
                                      monkeypatch):
    """Every job against the oracle, both precisions; queue "1" forces the
    persistent count kernel (tiles costliest first), None lets the
    autotuner choose."""
    if queue is not None:
        monkeypatch.setenv("C3X_BATCH_QUEUE", queue)
    raA, decA, raB, decB, jobs = batch_data
    print(f"[gpu] batch jobs={len(jobs)} precision={precision} queue={queue}", flush=True)
    b = c3x.Batch(jobs, _t(raA, dev), _t(decA, dev), _t(raB, dev), _t(decB, dev),
                  precision=precision)
    r0 = b.result()
    offs = b.pair_offsets()
    check_batch(r0, offs, jobs, batch_oracle)
    # graph replays: identical output
    for _ in range(2):
        b.run()
        r1 = b.result()
        assert np.array_equal(r1.idxA.cpu().numpy(), r0.idxA.cpu().numpy())
        assert np.array_equal(r1.idxB.cpu().numpy(), r0.idxB.cpu().numpy())
        assert np.array_equal(r1.sep.cpu().numpy(), r0.sep.cpu().numpy())
        assert np.array_equal(r1.best_idx.cpu().numpy(), r0.best_idx.cpu().numpy())
    st = b.stats()
    assert st["n_pairs"] == offs[-1] and st["n_tests"] > 0
    if queue is not None:
        assert st["queue"] == int(queue)
    b.free()


@pytest.mark.parametrize("scale", ["0.5", "3"])
def test_batch_fixed_cell_scales(c3x, dev, batch_data, batch_oracle, scale, monkeypatch):
    """Any cell scale gives the same answer (the autotuner only picks speed)."""
    monkeypatch.setenv("C3X_BATCH_CELL_SCALE", scale)
    raA, decA, raB, decB, jobs = batch_data
    b = c3x.Batch(jobs, _t(raA, dev), _t(decA, dev), _t(raB, dev), _t(decB, dev),
                  precision=1)
    check_batch(b.result(), b.pair_offsets(), jobs, batch_oracle)
    b.free()


def test_batch_cfg4_sample(c3x, dev):
    """A scaled-down draw of the 4,096-job workload (generator of the
    benchmark), checked job by job."""
    import oracle
    cat = synth.cfg4_jobs(scale=0.02)
    jobs = [tuple(int(v) for v in r[:4]) + (float(r[4]),) for r in cat.jobs]
    b = c3x.Batch(jobs, _t(cat.raA, dev), _t(cat.decA, dev), _t(cat.raB, dev), _t(cat.decB, dev),
                  precision=1)
    ors = [oracle.match(cat.raA[ao:ao + na], cat.decA[ao:ao + na], cat.raB[bo:bo + nb],
                        cat.decB[bo:bo + nb], radius_arcsec=r) for ao, na, bo, nb, r in jobs]
    check_batch(b.result(), b.pair_offsets(), jobs, ors)
    b.free()


def test_batch_errors(c3x, dev):
    ra = _t([10.0, 40.0], dev)
    de = _t([0.0, 0.0], dev)
    with pytest.raises(c3x.C3XError) as ei:
        c3x.Batch([(0, 2, 0, 2, 1.0)], ra, de, ra, de)
    assert "deg from their mean" in str(ei.value)
    bad = _t([10.0, float("nan")], dev)
    with pytest.raises(c3x.C3XError):
        c3x.Batch([(0, 2, 0, 2, 1.0)], bad, de, ra, de)


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_rows_with_thousands_of_matches(c3x, dev, precision):
    """A job whose sources hold tens of thousands of matches each (ordered
    after the graph by one segmented sort, then renumbered job-locally),
    beside ordinary jobs; every job against the oracle, and a replay."""
    import oracle
    g = np.random.default_rng(31)
    rb, db = synth.cap_uniform(g, 120_000, 40.0, -30.0, 0.3)
    ra, da = synth.cap_uniform(g, 10, 40.0, -30.0, 0.05)
    raA2, decA2, raB2, decB2, jobs2 = small_batch(seed=6)
    raA = np.concatenate([raA2, ra])
    decA = np.concatenate([decA2, da])
    raB = np.concatenate([raB2, rb])
    decB = np.concatenate([decB2, db])
    jobs = list(jobs2) + [(len(raA2), len(ra), len(raB2), len(rb), 400.0)]
    ors = [oracle.match(raA[ao:ao + na], decA[ao:ao + na], raB[bo:bo + nb], decB[bo:bo + nb],
                        radius_arcsec=r) for ao, na, bo, nb, r in jobs]
    assert np.bincount(ors[-1].ia).max() > 2048
    print(f"[gpu] batch long rows precision={precision}", flush=True)
    b = c3x.Batch(jobs, _t(raA, dev), _t(decA, dev), _t(raB, dev), _t(decB, dev),
                  precision=precision)
    check_batch(b.result(), b.pair_offsets(), jobs, ors)
    b.run()
    check_batch(b.result(), b.pair_offsets(), jobs, ors)
    b.free()


def _result_bytes(b):
    r = b.result()
    return [t.cpu().numpy().tobytes() for t in (r.idxA, r.idxB, r.sep, r.best_idx, r.best_sep)]


@pytest.mark.parametrize("name,value", [("C3X_BATCH_TILE", "64"), ("C3X_BATCH_TILE", "128"),
                                        ("C3X_BATCH_TILE", "256"), ("C3X_BATCH_QUEUE", "0"),
                                        ("C3X_BATCH_QUEUE", "1"),
                                        ("C3X_BATCH_CELL_SCALES", "0.5,4,1,2"),
                                        ("C3X_BATCH_CELL_SCALES", "4,0.5,2,0.5")])
def test_batch_autotuner_choices_give_identical_bytes(c3x, dev, name, value, monkeypatch):
    """Every setting the autotuner may pick -- the count kernel's tile, a
    cell scale per density class of job -- gives byte-identical outputs;
    the default (autotuned) run reports the tile it chose."""
    raA, decA, raB, decB, jobs = small_batch(seed=12)
    # jobs in every density class: add two larger ones
    g = np.random.default_rng(13)
    extra = []
    for n in (6_000, 50_000):
        ra, de = synth.cap_uniform(g, n, 120.0, -40.0, 0.5)
        rb, db = synth.cap_uniform(g, 10 * n, 120.0, -40.0, 0.5)
        extra.append((ra, de, rb, db))
    for ra, de, rb, db in extra:
        jobs.append((len(raA), len(ra), len(raB), len(rb), 3.0))
        raA, decA = np.concatenate([raA, ra]), np.concatenate([decA, de])
        raB, decB = np.concatenate([raB, rb]), np.concatenate([decB, db])
    t = [_t(x, dev) for x in (raA, decA, raB, decB)]
    b0 = c3x.Batch(jobs, *t, precision=1)
    want = _result_bytes(b0)
    assert b0.stats()["tile"] in (64, 128, 256)
    b0.free()
    monkeypatch.setenv(name, value)
    print(f"[gpu] batch {name}={value}", flush=True)
    b = c3x.Batch(jobs, *t, precision=1)
    assert _result_bytes(b) == want
    if name == "C3X_BATCH_TILE":
        assert b.stats()["tile"] == int(value)
    if name == "C3X_BATCH_QUEUE":
        assert b.stats()["queue"] == int(value)
    b.run()
    assert _result_bytes(b) == want
    b.free()
