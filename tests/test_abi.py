"""Host-side checks of libc3x.so that need no GPU: the library loads, exports
every function include/c3x.h declares, rejects bad arguments before touching
the device, and its binary128 fallback decides the closed-form cases right."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "c3x.h")


def header_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(c3x_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def L():
    import paper_1611_08494_amd as c3x
    return c3x.lib()


def test_header_declares_the_boundary():
    fns = header_functions()
    for f in ("c3x_build_index", "c3x_match", "c3x_result_sizes", "c3x_result_copy",
              "c3x_result_views", "c3x_result_stats", "c3x_result_free", "c3x_index_free", "c3x_last_error",
              "c3x_version", "c3x_abi_version", "c3x_index_stats", "c3x_result_unmatched",
              "c3x_match_concentric", "c3x_result_levels", "c3x_result_mutual",
              "c3x_cross_match"):
        assert f in fns


def test_every_declared_symbol_is_exported(L):
    for f in header_functions():
        assert hasattr(L, f), f


def test_version(L):
    assert L.c3x_abi_version() == 2
    assert b"gfx950" in L.c3x_version()


def test_argument_errors_need_no_device(L):
    from paper_1611_08494_amd import _binding as b
    h = ctypes.c_void_p()
    assert L.c3x_build_index(None, None, -1, 0, 1.0, None, ctypes.byref(h)) == b.EINVAL
    assert h.value is None
    assert b"nB < 0" in L.c3x_last_error()
    assert L.c3x_build_index(None, None, 1 << 31, 0, 1.0, None, ctypes.byref(h)) == b.ERANGE
    assert L.c3x_build_index(None, None, 5, 0, 1.0, None, ctypes.byref(h)) == b.EINVAL
    assert L.c3x_build_index(None, None, 0, 7, 1.0, None, ctypes.byref(h)) == b.EINVAL
    assert L.c3x_build_index(None, None, 0, 0, -1.0, None, ctypes.byref(h)) == b.EINVAL
    area = b.Area(shape=0, radius_arcsec=1.0, pa_sense=1)
    assert L.c3x_match(None, None, None, 0, 0, ctypes.byref(area), 3, None,
                       ctypes.byref(h)) == b.EINVAL
    assert L.c3x_result_sizes(None, None, None) == b.EINVAL
    b.lib()  # argument types
    assert L.c3x_result_views(None, None, None, None, None, None) == b.EINVAL
    assert L.c3x_result_unmatched(None, 1, None, None, None, None, None) == b.EINVAL
    assert L.c3x_match_concentric(None, None, None, 0, 0, None, None, 0, 1, None, None) == b.EINVAL
    h2 = ctypes.c_void_p()
    assert L.c3x_match_concentric(None, None, None, 0, 0, None, None, 0, 1, None,
                                  ctypes.byref(h2)) == b.EINVAL
    assert h2.value is None
    assert L.c3x_result_levels(None, None) == b.EINVAL
    h3, h4 = ctypes.c_void_p(), ctypes.c_void_p()
    assert L.c3x_cross_match(None, None, 0, 0, 1.0, None, None, 0, 0, ctypes.byref(area), 3,
                             None, ctypes.byref(h3), None) == b.EINVAL  # out NULL
    assert L.c3x_cross_match(None, None, -1, 0, 1.0, None, None, 0, 0, ctypes.byref(area), 3,
                             None, ctypes.byref(h3), ctypes.byref(h4)) == b.EINVAL
    assert b"nB < 0" in L.c3x_last_error()
    assert L.c3x_cross_match(None, None, 0, 0, 1.0, None, None, 5, 0, ctypes.byref(area), 3,
                             None, ctypes.byref(h3), ctypes.byref(h4)) == b.EINVAL
    assert L.c3x_cross_match(None, None, 0, 0, 1.0, None, None, 0, 0, None, 3,
                             None, ctypes.byref(h3), ctypes.byref(h4)) == b.EINVAL
    assert L.c3x_cross_match(None, None, 0, 9, 1.0, None, None, 0, 0, ctypes.byref(area), 3,
                             None, ctypes.byref(h3), ctypes.byref(h4)) == b.EINVAL
    assert h3.value is None and h4.value is None
    L.c3x_result_free(None)  # a no-op


def test_batch_argument_errors_need_no_device(L):
    from paper_1611_08494_amd import _binding as b
    b.lib()  # argument types
    h = ctypes.c_void_p()
    jobs = (b.Job * 2)(b.Job(0, 10, 0, 10, 1.0), b.Job(10, 5, 10, 5, 1.0))
    assert L.c3x_batch_plan(jobs, 0, None, None, None, None, 0, None, ctypes.byref(h)) == b.EINVAL
    assert h.value is None
    bad = (b.Job * 1)(b.Job(-1, 10, 0, 10, 1.0))
    assert L.c3x_batch_plan(bad, 1, None, None, None, None, 0, None, ctypes.byref(h)) == b.EINVAL
    assert b"negative" in L.c3x_last_error()
    wide = (b.Job * 1)(b.Job(0, 10, 0, 10, 7200.0))
    assert L.c3x_batch_plan(wide, 1, None, None, None, None, 0, None, ctypes.byref(h)) == b.EINVAL
    assert b"radius" in L.c3x_last_error()
    big = (b.Job * 2)(b.Job(0, 1 << 30, 0, 1, 1.0), b.Job(0, 1 << 30, 0, 1, 1.0))
    assert L.c3x_batch_plan(big, 2, None, None, None, None, 0, None, ctypes.byref(h)) == b.ERANGE
    assert L.c3x_batch_plan(jobs, 2, None, None, None, None, 0, None, ctypes.byref(h)) == b.EINVAL
    assert b"NULL" in L.c3x_last_error()
    assert L.c3x_batch_run(None, None) == b.EINVAL
    assert L.c3x_batch_result(None, None) == b.EINVAL


def _q(L):
    L.c3x_q_circle.argtypes = [ctypes.c_double] * 5
    L.c3x_q_circle.restype = ctypes.c_int
    L.c3x_q_ellipse.argtypes = [ctypes.c_double] * 8 + [ctypes.c_int]
    L.c3x_q_ellipse.restype = ctypes.c_int
    return L


def test_binary128_fallback_closed_forms(L):
    """The host fallback alone (no FP64 ladder in front) gets every
    closed-form case of tests/golden right."""
    from test_oracle_pins import CLOSED
    Q = _q(L)
    bad = []
    for r in CLOSED:
        if r["shape"] == 0:
            got = Q.c3x_q_circle(r["raA"], r["decA"], r["raB"], r["decB"], r["r"])
        else:
            got = Q.c3x_q_ellipse(r["raA"], r["decA"], r["raB"], r["decB"], r["a"], r["b"],
                                  r["pa"], r["pz"], r["sense"])
        if bool(got) != r["inside"]:
            bad.append(r)
    assert not bad, bad[:3]


def test_binary128_thresholds(L):
    L.c3x_q_thresholds.argtypes = [ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_double)]
    h = ctypes.c_double()
    c = ctypes.c_double()
    for r in (1e-6, 0.5, 1.0, 2.0, 60.0, 3600.0, 324000.0):
        L.c3x_q_thresholds(r, ctypes.byref(h), ctypes.byref(c))
        s = math.sin(r / 7200.0 * math.pi / 180.0)
        assert h.value == pytest.approx(s * s, rel=1e-14)
        assert c.value == pytest.approx(4 * s * s, rel=1e-14)


def test_binary128_against_200bit_on_near_boundary_pairs(L):
    """Random pairs placed within 2^-45 of the circle: binary128 and the
    oracle's 200-bit decider agree on every one."""
    import synth
    from oracle import exact
    Q = _q(L)
    c = synth.adversarial_circle(radius_arcsec=2.0, n_centres=16)
    n = c.nA
    for k in range(c.nB):
        i = k % n
        want = exact.decide_circle(c.raA[i], c.decA[i], c.raB[k], c.decB[k], 2.0)
        assert bool(Q.c3x_q_circle(c.raA[i], c.decA[i], c.raB[k], c.decB[k], 2.0)) == want


def test_binary128_best_against_200bit(L):
    """The host best-match ranking (FP64 pre-pass + binary128) returns the
    oracle's 200-bit argmin of (theta, index) on candidate sets built around
    exact ties (mirror images in Dec about the equator, in RA about the
    0/360 seam and through the pole) and one-ulp near-ties, mixed with
    random far candidates and shuffled."""
    from oracle import exact
    L.c3x_q_best.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int,
                             ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                             ctypes.POINTER(ctypes.c_int32)]
    L.c3x_q_best.restype = ctypes.c_int
    rng = np.random.default_rng(20240611)
    up = lambda x: float(np.nextafter(x, np.inf))
    dn = lambda x: float(np.nextafter(x, -np.inf))
    cases = []
    for e in (1e-4, 3e-4, 5.5e-4):
        cases.append((0.0, 0.0, [(e, 0.0), (360.0 - e, 0.0), (0.0, e), (0.0, -e)]))
        cases.append((0.0, 0.0, [(e, 0.0), (360.0 - e, 0.0), (0.0, up(e)), (0.0, -dn(e))]))
        cases.append((123.25, 0.0, [(123.25, e), (123.25, -e), (123.25 + e, 0.0)]))
        cases.append((10.0, 90.0, [(0.0, 90.0 - e), (180.0, 90.0 - e), (77.0, up(90.0 - e))]))
        cases.append((200.0, -45.0, [(200.0 + e, -45.0), (dn(200.0 + e), -45.0),
                                     (200.0, -45.0 + e)]))
    bad = []
    for ra1, dec1, near in cases:
        for trial in range(6):
            far = [(float((ra1 + rng.uniform(-0.01, 0.01)) % 360.0),
                    float(np.clip(dec1 + rng.uniform(-0.01, 0.01), -90, 90)))
                   for _ in range(rng.integers(0, 5))]
            pts = near + far
            idx = rng.permutation(len(pts) * 3)[:len(pts)].astype(np.int32)
            order = rng.permutation(len(pts))
            r2 = np.array([pts[k][0] for k in order], dtype=np.float64)
            d2 = np.array([pts[k][1] for k in order], dtype=np.float64)
            ib = np.ascontiguousarray(idx[order])
            k = L.c3x_q_best(ra1, dec1, len(pts),
                             r2.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             d2.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             ib.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
            want = exact.best_of(ra1, dec1, [(int(ib[q]), r2[q], d2[q]) for q in range(len(pts))])
            if int(ib[k]) != want:
                bad.append((ra1, dec1, pts, int(ib[k]), want))
    assert not bad, bad[:3]


def test_bench_reports_traffic_only_for_the_measured_kernel(monkeypatch):
    """roofline.traffic comes from the committed counter summary only while
    the count kernel's sources are the ones it was measured on."""
    import bench
    for cfg in ("cfg2", "cfg5"):
        got = bench.committed_traffic(cfg, "mixed")
        if got is not None:  # the summary matches the sources as committed
            assert got > 0
    assert bench.committed_traffic("cfg1", "mixed") is None
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: "0" * 16)
    for cfg in ("cfg2", "cfg5"):
        assert bench.committed_traffic(cfg, "mixed") is None
        assert bench.committed_traffic(cfg, "fp64") is None


def test_frame_rotation_matches_the_oracle(L):
    """The library's rotation of the frame conversion rule (binary128, host)
    equals the oracle's (200-bit mpmath) entry for entry, bit for bit."""
    import numpy as np
    from oracle import frames
    for src, dst in ((0, 1), (1, 0), (0, 0), (1, 1)):
        out = (ctypes.c_double * 9)()
        L.c3x_frame_matrix(src, dst, out)
        assert np.array_equal(np.array(list(out)), frames.rotation(src, dst)), (src, dst)
