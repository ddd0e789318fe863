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


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_matches_oracle_per_job(c3x, dev, batch_data, batch_oracle, precision):
    raA, decA, raB, decB, jobs = batch_data
    print(f"[gpu] batch jobs={len(jobs)} precision={precision}", flush=True)
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
