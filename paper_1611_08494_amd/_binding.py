"""ctypes binding of libc3x.so (declared in include/c3x.h).

Argument marshalling only: every step of the cross-match runs in the HIP
library. torch supplies device memory (float64 CUDA tensors on the current
device) and the stream the library orders its work on. If the library is not
built the import fails loudly; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_build", "libc3x.so")

OK, EINVAL, ERANGE, ENOMEM, EDEVICE, EFRAME = range(6)
EQUATORIAL, GALACTIC = 0, 1
CIRCLE, ELLIPSE, RECT = 0, 1, 2
ALL, BEST = 1, 2
FP64, MIXED = 0, 1
_STATUS = {0: "C3X_OK", 1: "C3X_EINVAL", 2: "C3X_ERANGE", 3: "C3X_ENOMEM", 4: "C3X_EDEVICE",
           5: "C3X_EFRAME"}


class C3XError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


class Area(ctypes.Structure):
    _fields_ = [
        ("shape", ctypes.c_int),
        ("radius_arcsec", ctypes.c_double),
        ("semi_major_arcsec", ctypes.c_void_p),
        ("semi_minor_arcsec", ctypes.c_void_p),
        ("pa_deg", ctypes.c_void_p),
        ("pa_zero_deg", ctypes.c_double),
        ("pa_sense", ctypes.c_int),
    ]


class Job(ctypes.Structure):
    _fields_ = [("a_off", ctypes.c_int64), ("nA", ctypes.c_int64), ("b_off", ctypes.c_int64),
                ("nB", ctypes.c_int64), ("radius_arcsec", ctypes.c_double)]


class Opts(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int),
        ("cell_arcsec", ctypes.c_double),
        ("tile", ctypes.c_int),
        ("stream", ctypes.c_void_p),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("n_a", ctypes.c_int64), ("n_b", ctypes.c_int64), ("n_pairs", ctypes.c_int64),
        ("n_tests", ctypes.c_int64), ("n_band", ctypes.c_int64),
        ("n_ambiguous", ctypes.c_int64), ("n_best_ties", ctypes.c_int64),
        ("n_cells", ctypes.c_int64), ("cell_arcsec", ctypes.c_double),
        ("ms_index", ctypes.c_double), ("ms_a_prep", ctypes.c_double),
        ("ms_count", ctypes.c_double), ("ms_scan", ctypes.c_double),
        ("ms_write", ctypes.c_double), ("ms_sort_pairs", ctypes.c_double),
        ("ms_total", ctypes.c_double), ("precision", ctypes.c_int32), ("tile", ctypes.c_int32),
        ("ms_count_kernel", ctypes.c_double),
        ("n_sort_retries", ctypes.c_int32),
        ("queue", ctypes.c_int32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def lib():
    """Loads libc3x.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(hipcc for gfx950); there is no CPU fallback")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    L.c3x_build_index.argtypes = [vp, vp, i64, ctypes.c_int, dbl, ctypes.POINTER(Opts),
                                  ctypes.POINTER(vp)]
    L.c3x_build_index.restype = ctypes.c_int
    L.c3x_match.argtypes = [vp, vp, vp, i64, ctypes.c_int, ctypes.POINTER(Area), ctypes.c_uint,
                            ctypes.POINTER(Opts), ctypes.POINTER(vp)]
    L.c3x_match.restype = ctypes.c_int
    L.c3x_result_sizes.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.c3x_result_sizes.restype = ctypes.c_int
    L.c3x_result_copy.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.c3x_result_copy.restype = ctypes.c_int
    pvp = ctypes.POINTER(vp)
    L.c3x_result_views.argtypes = [vp, pvp, pvp, pvp, pvp, pvp]
    L.c3x_result_views.restype = ctypes.c_int
    L.c3x_result_unmatched.argtypes = [vp, ctypes.c_uint, vp, pvp, ctypes.POINTER(i64), pvp,
                                       ctypes.POINTER(i64)]
    L.c3x_match_concentric.argtypes = [vp, vp, vp, i64, ctypes.c_int, ctypes.POINTER(Area),
                                       ctypes.POINTER(dbl), i32, ctypes.c_uint,
                                       ctypes.POINTER(Opts), ctypes.POINTER(vp)]
    L.c3x_match_concentric.restype = ctypes.c_int
    L.c3x_cross_match.argtypes = [vp, vp, i64, ctypes.c_int, dbl, vp, vp, i64, ctypes.c_int,
                                  ctypes.POINTER(Area), ctypes.c_uint, ctypes.POINTER(Opts),
                                  ctypes.POINTER(vp), ctypes.POINTER(vp)]
    L.c3x_cross_match.restype = ctypes.c_int
    L.c3x_result_mutual.argtypes = [vp, vp, vp, vp, vp, vp, pvp, pvp, pvp, ctypes.POINTER(i64),
                                    pvp]
    L.c3x_result_mutual.restype = ctypes.c_int
    L.c3x_frame_convert.argtypes = [vp, vp, i64, ctypes.c_int, ctypes.c_int, vp, vp, vp, vp]
    L.c3x_frame_convert.restype = ctypes.c_int
    L.c3x_frame_matrix.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(dbl)]
    L.c3x_frame_matrix.restype = None
    L.c3x_exact_match.argtypes = [vp, i64, vp, i64, ctypes.c_int, ctypes.c_uint, vp,
                                  ctypes.POINTER(vp)]
    L.c3x_exact_match.restype = ctypes.c_int
    L.c3x_result_levels.argtypes = [vp, pvp]
    L.c3x_result_levels.restype = ctypes.c_int
    L.c3x_result_unmatched.restype = ctypes.c_int
    L.c3x_result_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    L.c3x_result_stats.restype = ctypes.c_int
    L.c3x_index_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    L.c3x_index_stats.restype = ctypes.c_int
    L.c3x_result_free.argtypes = [vp]
    L.c3x_result_free.restype = None
    L.c3x_index_free.argtypes = [vp]
    L.c3x_index_free.restype = None
    L.c3x_batch_plan.argtypes = [ctypes.POINTER(Job), i32, vp, vp, vp, vp, ctypes.c_int,
                                 ctypes.POINTER(Opts), ctypes.POINTER(vp)]
    L.c3x_batch_plan.restype = ctypes.c_int
    L.c3x_batch_run.argtypes = [vp, vp]
    L.c3x_batch_run.restype = ctypes.c_int
    L.c3x_batch_result.argtypes = [vp, ctypes.POINTER(vp)]
    L.c3x_batch_result.restype = ctypes.c_int
    L.c3x_batch_offsets.argtypes = [vp, ctypes.POINTER(i64)]
    L.c3x_batch_offsets.restype = ctypes.c_int
    L.c3x_batch_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    L.c3x_batch_stats.restype = ctypes.c_int
    L.c3x_batch_free.argtypes = [vp]
    L.c3x_batch_free.restype = None
    L.c3x_last_error.restype = ctypes.c_char_p
    L.c3x_version.restype = ctypes.c_char_p
    L.c3x_abi_version.restype = ctypes.c_int
    _lib = L
    return L


def check(status: int):
    if status != OK:
        raise C3XError(status, lib().c3x_last_error().decode())


def _torch():
    import torch
    return torch


def _dev_f64(t, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != torch.float64 or not t.is_contiguous() or t.dim() != 1:
        raise TypeError(f"{name} must be a contiguous 1-D float64 tensor")
    return t


def _stream_ptr(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Index:
    """Immutable sky index over catalogue B (owns its device buffers)."""

    def __init__(self, handle, n, frame, precision):
        self._h = handle
        self.n = n
        self.frame = frame
        self.precision = precision

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("index was freed")
        return self._h

    def stats(self) -> dict:
        s = Stats()
        check(lib().c3x_index_stats(self.handle, ctypes.byref(s)))
        return s.as_dict()

    def free(self):
        if self._h is not None:
            lib().c3x_index_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class MatchResult:
    def __init__(self, idxA, idxB, sep, best_idx, best_sep, stats, owner=None):
        self.idxA = idxA
        self.idxB = idxB
        self.sep = sep
        self.best_idx = best_idx
        self.best_sep = best_sep
        self.stats = stats
        self._owner = owner  # the c3x_result behind the views

    @property
    def n_pairs(self) -> int:
        return int(self.idxA.shape[0])


def build_index(ra, dec, frame: int = EQUATORIAL, reach_hint_arcsec: float = 0.0,
                precision: int = FP64, cell_arcsec: float = 0.0, stream=None) -> Index:
    ra = _dev_f64(ra, "ra")
    dec = _dev_f64(dec, "dec")
    if ra.shape != dec.shape:
        raise ValueError("ra and dec differ in length")
    o = Opts(precision=int(precision), cell_arcsec=float(cell_arcsec), tile=0,
             stream=_stream_ptr(stream))
    h = ctypes.c_void_p()
    check(lib().c3x_build_index(ra.data_ptr(), dec.data_ptr(), ra.shape[0], int(frame),
                                float(reach_hint_arcsec), ctypes.byref(o), ctypes.byref(h)))
    return Index(h, ra.shape[0], frame, precision)


class _ResultOwner:
    """Keeps a c3x_result alive while tensors view its device arrays."""

    def __init__(self, handle):
        self.handle = handle

    def __del__(self):
        if self.handle:
            lib().c3x_result_free(self.handle)
            self.handle = None


class _DeviceArray:
    """One of a result's arrays, exposed without a copy (CUDA array interface;
    the tensor made from it keeps it, and so the result, alive)."""

    def __init__(self, owner, ptr, n, typestr):
        self.owner = owner
        self.__cuda_array_interface__ = {"shape": (n,), "typestr": typestr,
                                         "data": (ptr, False), "version": 2}


def _views(h, dev) -> MatchResult:
    """Tensors over the result's own device arrays; the result is freed when
    the last of them goes."""
    torch = _torch()
    owner = _ResultOwner(h)
    npairs = ctypes.c_int64()
    na = ctypes.c_int64()
    check(lib().c3x_result_sizes(h, ctypes.byref(npairs), ctypes.byref(na)))
    ptrs = [ctypes.c_void_p() for _ in range(5)]
    check(lib().c3x_result_views(h, *[ctypes.byref(p) for p in ptrs]))
    st = Stats()
    check(lib().c3x_result_stats(h, ctypes.byref(st)))
    out = []
    for p, n, ts, dt in zip(ptrs, (npairs.value,) * 3 + (na.value,) * 2,
                            ("<i4", "<i4", "<f8", "<i4", "<f8"),
                            (torch.int32, torch.int32, torch.float64, torch.int32,
                             torch.float64)):
        if n == 0 or not p.value:
            out.append(torch.empty(n, dtype=dt, device=dev))
        else:
            out.append(torch.as_tensor(_DeviceArray(owner, p.value, n, ts), device=dev))
    return MatchResult(*out, st.as_dict(), owner=owner)


def match(index: Index, ra, dec, frame: int = EQUATORIAL, shape: int = CIRCLE,
          radius_arcsec: float = 1.0, a=None, b=None, pa=None, pa_zero_deg: float = 0.0,
          pa_sense: int = 1, mode: int = ALL | BEST, stream=None) -> MatchResult:
    """Cross-matches catalogue A (ra, dec) against ``index``. Returns device
    tensors: idxA, idxB (int32), sep (float64 arcsec) in canonical order and
    best_idx (int32, -1 if unmatched), best_sep (float64, NaN) per A row.
    The tensors view the result's own device arrays (no copy)."""
    ra = _dev_f64(ra, "ra")
    dec = _dev_f64(dec, "dec")
    if ra.shape != dec.shape:
        raise ValueError("ra and dec differ in length")
    ar = Area(shape=int(shape), radius_arcsec=float(radius_arcsec), pa_zero_deg=float(pa_zero_deg),
              pa_sense=int(pa_sense))
    if shape in (ELLIPSE, RECT):
        for nm, v in (("a", a), ("b", b), ("pa", pa)):
            v = _dev_f64(v, nm)
            if v.shape != ra.shape:
                raise ValueError(f"{nm} must have one entry per A row")
        ar.semi_major_arcsec = a.data_ptr()
        ar.semi_minor_arcsec = b.data_ptr()
        ar.pa_deg = pa.data_ptr()
    sp = _stream_ptr(stream)
    o = Opts(precision=int(index.precision), cell_arcsec=0.0, tile=0, stream=sp)
    h = ctypes.c_void_p()
    check(lib().c3x_match(index.handle, ra.data_ptr(), dec.data_ptr(), ra.shape[0], int(frame),
                          ctypes.byref(ar), int(mode), ctypes.byref(o), ctypes.byref(h)))
    return _views(h, ra.device)


def cross_match(raB, decB, raA, decA, frame: int = EQUATORIAL, frameA: int = None,
                reach_hint_arcsec: float = 0.0, precision: int = FP64, cell_arcsec: float = 0.0,
                shape: int = CIRCLE, radius_arcsec: float = 1.0, a=None, b=None, pa=None,
                pa_zero_deg: float = 0.0, pa_sense: int = 1, mode: int = ALL | BEST,
                keep_index: bool = False, stream=None):
    """The index over catalogue B and the match of catalogue A in one call
    (c3x_cross_match): what ``build_index`` then ``match`` return, with A
    keyed and sorted while B's index is built. ``frame`` is B's frame
    (``frameA``: A's, default the same). Returns the MatchResult, or
    (MatchResult, Index) with ``keep_index``."""
    raB = _dev_f64(raB, "raB")
    decB = _dev_f64(decB, "decB")
    ra = _dev_f64(raA, "raA")
    dec = _dev_f64(decA, "decA")
    if raB.shape != decB.shape or ra.shape != dec.shape:
        raise ValueError("ra and dec differ in length")
    ar = Area(shape=int(shape), radius_arcsec=float(radius_arcsec), pa_zero_deg=float(pa_zero_deg),
              pa_sense=int(pa_sense))
    if shape in (ELLIPSE, RECT):
        for nm, v in (("a", a), ("b", b), ("pa", pa)):
            v = _dev_f64(v, nm)
            if v.shape != ra.shape:
                raise ValueError(f"{nm} must have one entry per A row")
        ar.semi_major_arcsec = a.data_ptr()
        ar.semi_minor_arcsec = b.data_ptr()
        ar.pa_deg = pa.data_ptr()
    o = Opts(precision=int(precision), cell_arcsec=float(cell_arcsec), tile=0,
             stream=_stream_ptr(stream))
    hi = ctypes.c_void_p()
    h = ctypes.c_void_p()
    fa = frame if frameA is None else frameA
    check(lib().c3x_cross_match(raB.data_ptr(), decB.data_ptr(), raB.shape[0], int(frame),
                                float(reach_hint_arcsec), ra.data_ptr(), dec.data_ptr(),
                                ra.shape[0], int(fa), ctypes.byref(ar), int(mode),
                                ctypes.byref(o), ctypes.byref(hi) if keep_index else None,
                                ctypes.byref(h)))
    r = _views(h, ra.device)
    if keep_index:
        return r, Index(hi, raB.shape[0], frame, precision)
    return r


def frame_matrix(src: int, dst: int):
    """The frame conversion rule's rotation (c3x_frame_matrix), 9 doubles
    row-major."""
    out = (ctypes.c_double * 9)()
    lib().c3x_frame_matrix(int(src), int(dst), out)
    return list(out)


def frame_convert(ra, dec, src: int, dst: int, stream=None):
    """Positions converted from frame src to frame dst by the library's fixed
    FP64 rule (c3x_frame_convert): device tensors (ra', dec', gamma), gamma
    the angle that turns an orientation from frame src into frame dst."""
    torch = _torch()
    ra = _dev_f64(ra, "ra")
    dec = _dev_f64(dec, "dec")
    if ra.shape != dec.shape:
        raise ValueError("ra and dec differ in length")
    out = [torch.empty_like(ra) for _ in range(3)]
    check(lib().c3x_frame_convert(ra.data_ptr(), dec.data_ptr(), ra.shape[0], int(src),
                                  int(dst), *[t.data_ptr() for t in out], _stream_ptr(stream)))
    return tuple(out)


KEY_I64, KEY_F64 = 0, 1


def exact_match(keyA, keyB, mode: int = ALL | BEST, stream=None) -> MatchResult:
    """The Exact Value case (c3x_exact_match): rows of A and B match when
    their key columns (1-D contiguous int64 or float64 CUDA tensors of one
    dtype) hold equal values. Returns the result like ``match`` (separations
    0, best_idx the lowest matching B row)."""
    torch = _torch()
    for t, nm in ((keyA, "keyA"), (keyB, "keyB")):
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dim() != 1 \
                or not t.is_contiguous() or t.dtype not in (torch.int64, torch.float64):
            raise TypeError(f"{nm} must be a contiguous 1-D int64 or float64 CUDA tensor")
    if keyA.dtype != keyB.dtype:
        raise TypeError("keyA and keyB must have one dtype")
    kt = KEY_I64 if keyA.dtype == torch.int64 else KEY_F64
    h = ctypes.c_void_p()
    check(lib().c3x_exact_match(keyA.data_ptr(), keyA.shape[0], keyB.data_ptr(), keyB.shape[0],
                                kt, int(mode), _stream_ptr(stream), ctypes.byref(h)))
    return _views(h, keyA.device)


def result_copy(result: MatchResult, idxA=None, idxB=None, sep=None, best_idx=None,
                best_sep=None, stream=None):
    """c3x_result_copy: copies the result's arrays into the given contiguous
    tensors (host or device; int32 idxA/idxB/best_idx, float64 sep/best_sep;
    n_pairs or nA entries). Any may be None."""
    torch = _torch()
    owner = result._owner
    if owner is None or not owner.handle:
        raise ValueError("result has no library handle")
    npairs, na = result.n_pairs, int(result.best_idx.shape[0])
    ptrs = []
    for t, n, dt, nm in ((idxA, npairs, torch.int32, "idxA"), (idxB, npairs, torch.int32, "idxB"),
                         (sep, npairs, torch.float64, "sep"),
                         (best_idx, na, torch.int32, "best_idx"),
                         (best_sep, na, torch.float64, "best_sep")):
        if t is None:
            ptrs.append(None)
            continue
        if t.dtype != dt or not t.is_contiguous() or t.numel() < n:
            raise TypeError(f"{nm} must be a contiguous {dt} tensor of at least {n} entries")
        ptrs.append(t.data_ptr())
    check(lib().c3x_result_copy(owner.handle, *ptrs, _stream_ptr(stream)))


def match_concentric(index: Index, ra, dec, a, b, pa, scales, frame: int = EQUATORIAL,
                     pa_zero_deg: float = 0.0, pa_sense: int = 1, mode: int = ALL | BEST,
                     stream=None) -> MatchResult:
    """Concentric ellipses (c3x_match_concentric): the result of the largest
    scaled ellipse, with ``level`` (int32 device tensor, one entry per pair):
    the index in ``scales`` (ascending) of the smallest ellipse holding the
    pair's B source."""
    torch = _torch()
    ra = _dev_f64(ra, "ra")
    dec = _dev_f64(dec, "dec")
    if ra.shape != dec.shape:
        raise ValueError("ra and dec differ in length")
    for nm, v in (("a", a), ("b", b), ("pa", pa)):
        if _dev_f64(v, nm).shape != ra.shape:
            raise ValueError(f"{nm} must have one entry per A row")
    ar = Area(shape=ELLIPSE, radius_arcsec=0.0, pa_zero_deg=float(pa_zero_deg),
              pa_sense=int(pa_sense))
    ar.semi_major_arcsec = a.data_ptr()
    ar.semi_minor_arcsec = b.data_ptr()
    ar.pa_deg = pa.data_ptr()
    ks = (ctypes.c_double * len(scales))(*[float(k) for k in scales])
    o = Opts(precision=int(index.precision), cell_arcsec=0.0, tile=0, stream=_stream_ptr(stream))
    h = ctypes.c_void_p()
    check(lib().c3x_match_concentric(index.handle, ra.data_ptr(), dec.data_ptr(), ra.shape[0],
                                     int(frame), ctypes.byref(ar), ks, len(scales), int(mode),
                                     ctypes.byref(o), ctypes.byref(h)))
    r = _views(h, ra.device)
    p = ctypes.c_void_p()
    check(lib().c3x_result_levels(r._owner.handle, ctypes.byref(p)))
    n = r.n_pairs
    r.level = (torch.as_tensor(_DeviceArray(r._owner, p.value, n, "<i4"), device=ra.device)
               if n and p.value else torch.empty(0, dtype=torch.int32, device=ra.device))
    return r


class Batch:
    """A planned batch of independent circular cross-matches (c3x_batch_*).
    ``jobs`` rows are (a_off, nA, b_off, nB, radius_arcsec). The input
    tensors are kept alive here: the batch reads them on every run."""

    def __init__(self, jobs, raA, decA, raB, decB, frame: int = EQUATORIAL,
                 precision: int = MIXED):
        self._keep = [_dev_f64(x, n) for x, n in ((raA, "raA"), (decA, "decA"), (raB, "raB"),
                                                    (decB, "decB"))]
        rows = [tuple(r) for r in jobs]
        self.n_jobs = len(rows)
        arr = (Job * max(1, self.n_jobs))()
        for k, (ao, na, bo, nb, r) in enumerate(rows):
            arr[k] = Job(int(ao), int(na), int(bo), int(nb), float(r))
        self._jobs = rows
        o = Opts(precision=int(precision), cell_arcsec=0.0, tile=0, stream=None)
        h = ctypes.c_void_p()
        ra_, de_, rb_, db_ = self._keep
        check(lib().c3x_batch_plan(arr, self.n_jobs, ra_.data_ptr(), de_.data_ptr(),
                                   rb_.data_ptr(), db_.data_ptr(), int(frame), ctypes.byref(o),
                                   ctypes.byref(h)))
        self._h = h
        self.device = ra_.device

    def run(self, stream=None):
        check(lib().c3x_batch_run(self._h, _stream_ptr(stream)))

    def result(self) -> MatchResult:
        h = ctypes.c_void_p()
        check(lib().c3x_batch_result(self._h, ctypes.byref(h)))
        return _views(h, self.device)

    def pair_offsets(self):
        out = (ctypes.c_int64 * (self.n_jobs + 1))()
        check(lib().c3x_batch_offsets(self._h, out))
        return list(out)

    def stats(self) -> dict:
        st = Stats()
        check(lib().c3x_batch_stats(self._h, ctypes.byref(st)))
        return st.as_dict()

    def free(self):
        if self._h:
            lib().c3x_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def unmatched(result: MatchResult, selection: int = ALL, stream=None):
    """Rows in no stored pair (c3x_result_unmatched): int32 device tensors of
    the unmatched A rows and the unmatched B rows, ascending. selection ALL
    stores every match, BEST each A row's best pair. The tensors view
    arrays owned by the result (a later call on it overwrites them)."""
    torch = _torch()
    owner = result._owner
    if owner is None or not owner.handle:
        raise ValueError("result has no library handle")
    pa, pb = ctypes.c_void_p(), ctypes.c_void_p()
    na, nb = ctypes.c_int64(), ctypes.c_int64()
    check(lib().c3x_result_unmatched(owner.handle, int(selection), _stream_ptr(stream),
                                     ctypes.byref(pa), ctypes.byref(na), ctypes.byref(pb),
                                     ctypes.byref(nb)))
    dev = result.best_idx.device
    out = []
    for p, n in ((pa, na.value), (pb, nb.value)):
        if n == 0 or not p.value:
            out.append(torch.empty(0, dtype=torch.int32, device=dev))
        else:
            out.append(torch.as_tensor(_DeviceArray(owner, p.value, n, "<i4"), device=dev))
    return out[0], out[1]


def mutual(result: MatchResult, raA, decA, raB, decB, stream=None):
    """Symmetric best pairs (c3x_result_mutual) of a result made with ALL |
    BEST, given the coordinate tensors of that match: int32 idxA, idxB and
    float64 sep of the pairs that are each other's nearest match (ascending
    A row), and best_a_of_b, the nearest A row of every B row (-1: none).
    The tensors view arrays owned by the result (a later call on it
    overwrites them)."""
    torch = _torch()
    owner = result._owner
    if owner is None or not owner.handle:
        raise ValueError("result has no library handle")
    ts = [_dev_f64(x, n) for x, n in ((raA, "raA"), (decA, "decA"), (raB, "raB"), (decB, "decB"))]
    pa, pb, ps, pbb = (ctypes.c_void_p() for _ in range(4))
    n = ctypes.c_int64()
    check(lib().c3x_result_mutual(owner.handle, *[t.data_ptr() for t in ts], _stream_ptr(stream),
                                  ctypes.byref(pa), ctypes.byref(pb), ctypes.byref(ps),
                                  ctypes.byref(n), ctypes.byref(pbb)))
    dev = result.best_idx.device
    out = []
    for p, m, ts_, dt in ((pa, n.value, "<i4", torch.int32), (pb, n.value, "<i4", torch.int32),
                          (ps, n.value, "<f8", torch.float64),
                          (pbb, int(ts[2].shape[0]), "<i4", torch.int32)):
        if m == 0 or not p.value:
            out.append(torch.empty(0 if p is not pbb else m, dtype=dt, device=dev))
        else:
            out.append(torch.as_tensor(_DeviceArray(owner, p.value, m, ts_), device=dev))
    return tuple(out)


# join type -> (stored pairs, unmatched A rows, unmatched B rows), Section 2.2
JOIN_PARTS = {
    "1and2": (True, False, False),
    "1or2": (True, True, True),
    "all1": (True, True, False),
    "all2": (True, False, True),
    "1not2": (False, True, False),
    "2not1": (False, False, True),
    "1xor2": (False, True, True),
}


def join(result: MatchResult, how: str, selection: int = ALL, stream=None) -> dict:
    """The rows of join type ``how`` (keys of JOIN_PARTS) as a dict of the
    parts it keeps (None for the parts it leaves out): the stored pairs --
    selection ALL: "idxA", "idxB", "sep" (every match); selection BEST:
    "best_idx", "best_sep" (A row a with best_idx[a] when >= 0) -- and the
    unmatched rows "rowsA", "rowsB". Only assembles what the result and
    c3x_result_unmatched hold."""
    if how not in JOIN_PARTS:
        raise ValueError(f"join must be one of {sorted(JOIN_PARTS)}")
    keep_p, keep_a, keep_b = JOIN_PARTS[how]
    ua, ub = unmatched(result, selection, stream)
    out = {"idxA": None, "idxB": None, "sep": None, "best_idx": None, "best_sep": None,
           "rowsA": ua if keep_a else None, "rowsB": ub if keep_b else None}
    if keep_p and selection == ALL:
        out.update(idxA=result.idxA, idxB=result.idxB, sep=result.sep)
    elif keep_p:
        out.update(best_idx=result.best_idx, best_sep=result.best_sep)
    return out


def version() -> str:
    return lib().c3x_version().decode()
