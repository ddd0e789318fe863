"""c3x_result_unmatched_noalloc, the form of c3x_result_unmatched that
allocates nothing (for callers that cannot allocate device memory), against
c3x_result_unmatched itself through the C ABI: two calls in a row on one
GPU, the second on a smaller result, both selections; the library's
allocator is armed to fail its next allocation during each call (a call
that allocated would fail); results above the fixed working memory are
refused with C3X_ERANGE; bad capacities with C3X_EINVAL."""
import ctypes

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
    L = m.lib()
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    L.c3x_result_unmatched_noalloc.argtypes = [vp, ctypes.c_uint, vp, vp, i64, vp, i64, vp]
    L.c3x_result_unmatched_noalloc.restype = ctypes.c_int
    L.c3x_debug_fail_alloc.argtypes = [ctypes.c_int]
    L.c3x_debug_fail_alloc.restype = None
    L.c3x_debug_live_blocks.restype = ctypes.c_int
    return m


def _t(x, dev):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64), device=dev)


def _noalloc(c3x, r, sel, nA, nB, dev):
    import torch
    L = c3x.lib()
    bufA = torch.full((max(nA, 1),), -7, dtype=torch.int32, device=dev)
    bufB = torch.full((max(nB, 1),), -7, dtype=torch.int32, device=dev)
    counts = torch.full((2,), -9, dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    live = L.c3x_debug_live_blocks()
    L.c3x_debug_fail_alloc(1)  # any allocation inside the call would fail it
    st = L.c3x_result_unmatched_noalloc(r._owner.handle, sel, None, bufA.data_ptr(), nA,
                                        bufB.data_ptr(), nB, counts.data_ptr())
    L.c3x_debug_fail_alloc(0)
    assert st == 0, L.c3x_last_error()
    torch.cuda.synchronize()
    assert L.c3x_debug_live_blocks() == live
    na, nb = counts.cpu().tolist()
    return bufA[:na].cpu().numpy(), bufB[:nb].cpu().numpy()


def test_two_calls_match_the_allocating_entry_point(c3x, dev):
    for scale in (0.004, 0.001):  # the second call on a smaller result
        cat = synth.cfg2_fullsky(scale=scale)
        print(f"[gpu] noalloc {cat.nA} x {cat.nB}", flush=True)
        ix = c3x.build_index(_t(cat.raB, dev), _t(cat.decB, dev), reach_hint_arcsec=2.0)
        r = c3x.match(ix, _t(cat.raA, dev), _t(cat.decA, dev), radius_arcsec=2.0,
                      mode=c3x.ALL | c3x.BEST)
        for sel in (c3x.ALL, c3x.BEST):
            ua, ub = (x.cpu().numpy().copy() for x in c3x.unmatched(r, sel))
            ga, gb = _noalloc(c3x, r, sel, cat.nA, cat.nB, dev)
            assert np.array_equal(ga, ua) and np.array_equal(gb, ub), (scale, sel)
            assert 0 < len(ua) < cat.nA and 0 < len(ub) < cat.nB
        ix.free()


def test_refusals(c3x, dev):
    import torch
    L = c3x.lib()
    g = torch.Generator(device=dev)
    g.manual_seed(5)
    n = 70_000_000  # nA + nB above what the fixed 64 MiB of working memory holds
    raB = torch.rand(n, generator=g, device=dev, dtype=torch.float64) * 359.0
    decB = torch.rand(n, generator=g, device=dev, dtype=torch.float64) * 170.0 - 85.0
    ix = c3x.build_index(raB, decB, reach_hint_arcsec=1.0)
    one = _t([10.0], dev)
    r = c3x.match(ix, one, one, radius_arcsec=1.0, mode=c3x.ALL | c3x.BEST)
    buf = torch.zeros(n, dtype=torch.int32, device=dev)
    counts = torch.zeros(2, dtype=torch.int64, device=dev)
    st = L.c3x_result_unmatched_noalloc(r._owner.handle, c3x.ALL, None, buf.data_ptr(), 1,
                                        buf.data_ptr(), n, counts.data_ptr())
    assert st == 2 and b"working memory" in L.c3x_last_error()  # C3X_ERANGE
    st = L.c3x_result_unmatched_noalloc(r._owner.handle, c3x.ALL, None, buf.data_ptr(), 0,
                                        buf.data_ptr(), n, counts.data_ptr())
    assert st == 1  # capacity below nA
    ix.free()
