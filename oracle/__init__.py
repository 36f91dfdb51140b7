"""CPU ORACLE for the KPA grouping path -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg use this package.  It never imports the GPU library and the GPU library
never imports it.  ``liboracle.so`` is built from ``oracle.cpp`` by
``oracle/build.py`` (plain g++ -O2, no intrinsics).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import mlp  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_u64 = C.c_uint64
_i = C.c_int
_u32 = C.c_uint32
_vp = C.c_void_p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from .build import build
            build()
        L = C.CDLL(LIB_PATH)
        L.orc_partition.argtypes = [_vp, _u64, _i, _i, _i, _i, _u64, _u64, _u32, _u64, _u64p, _u32p,
                                    _u64p, _u64p]
        L.orc_extract.argtypes = [_vp, _u64, _i, _i, _u64, _u64p, _u32p]
        L.orc_sort.argtypes = [_u64p, _u32p, _u64, _u64p, _u32p]
        L.orc_sort_segmented.argtypes = [_u64p, _u32p, _u64p, _u32, _u64p, _u32p]
        L.orc_merge.argtypes = [_u64p, _u32p, _u64, _u64p, _u32p, _u64, _u64p, _u32p]
        L.orc_reduce_by_key.argtypes = [_u64p, _u32p, _u64, _vp, _i, _i, _i, _u64p, _u64p, _u64p,
                                        _u64p, _u64p]
        L.orc_topk_by_sum.argtypes = [_u64p, _u64p, _u64, _u32, _u64p, _u64p, C.POINTER(_u32)]
        L.orc_median_by_key.argtypes = [_u64p, _u32p, _u64, _vp, _i, _i, _i, _u64p, _u64p, _u64p]
        L.orc_join.argtypes = [_u64p, _u32p, _u64, _u64p, _u32p, _u64, _vp, _vp, _i, _i, _i, _u64p,
                               _u64p, _vp, _u64, _u64p]
        L.orc_materialize.argtypes = [_u32p, _u64, _vp, _i, _vp]
        L.orc_pwl_fit.argtypes = [_u64p, _u64, _u32, _u64p, _u64p, _f32p]
        L.orc_window_aggregate.argtypes = [_vp, _u64, _i, _i, _i, _i, _i, _i, _u64, _u64, _u32,
                                           _u32, _i, _u64p, _u64p, _u64p, _u64p]
        for f in ("orc_partition", "orc_extract", "orc_sort", "orc_sort_segmented", "orc_merge",
                  "orc_reduce_by_key", "orc_topk_by_sum", "orc_median_by_key", "orc_join",
                  "orc_materialize", "orc_pwl_fit", "orc_window_aggregate"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _rows_np(rows) -> np.ndarray:
    """Rows as a C-contiguous byte-addressable numpy array (host)."""
    if hasattr(rows, "detach"):
        rows = rows.detach().cpu().numpy()
    rows = np.ascontiguousarray(rows)
    return rows


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _u64a(x):
    if hasattr(x, "detach"):
        x = x.detach().cpu().numpy()
    x = np.asarray(x)
    if x.dtype == np.int64:
        x = x.view(np.uint64)
    return np.ascontiguousarray(x, dtype=np.uint64)


def _u32a(x):
    if hasattr(x, "detach"):
        x = x.detach().cpu().numpy()
    x = np.asarray(x)
    if x.dtype == np.int32:
        x = x.view(np.uint32)
    return np.ascontiguousarray(x, dtype=np.uint32)


def _ck(rc):
    if rc != 0:
        raise ValueError(f"oracle call failed: {rc}")


def partition(rows, layout, win_len, n_win, origin=0, rid_base=0):
    r = _rows_np(rows)
    n = r.nbytes // layout.row_bytes
    keys = np.empty(n, np.uint64); rids = np.empty(n, np.uint32)
    off = np.empty(n_win + 1, np.uint64); oob = np.zeros(1, np.uint64)
    _ck(lib().orc_partition(_ptr(r), n, layout.row_bytes, layout.key_off, layout.ts_off,
                            layout.ts_w, win_len, origin, n_win, rid_base, keys, rids, off, oob))
    m = int(off[-1])
    return keys[:m], rids[:m], off, int(oob[0])


def extract(rows, layout, rid_base=0):
    r = _rows_np(rows)
    n = r.nbytes // layout.row_bytes
    keys = np.empty(n, np.uint64); rids = np.empty(n, np.uint32)
    _ck(lib().orc_extract(_ptr(r), n, layout.row_bytes, layout.key_off, rid_base, keys, rids))
    return keys, rids


def sort(keys, rids):
    k = _u64a(keys); r = _u32a(rids)
    ok = np.empty_like(k); orr = np.empty_like(r)
    _ck(lib().orc_sort(k, r, k.shape[0], ok, orr))
    return ok, orr


def sort_segmented(keys, rids, seg_off):
    k = _u64a(keys); r = _u32a(rids); s = _u64a(seg_off)
    ok = k.copy(); orr = r.copy()
    _ck(lib().orc_sort_segmented(k, r, s, s.shape[0] - 1, ok, orr))
    return ok, orr


def merge(ak, ar, bk, br):
    ak = _u64a(ak); ar = _u32a(ar); bk = _u64a(bk); br = _u32a(br)
    ok = np.empty(ak.shape[0] + bk.shape[0], np.uint64); orr = np.empty(ok.shape[0], np.uint32)
    _ck(lib().orc_merge(ak, ar, ak.shape[0], bk, br, bk.shape[0], ok, orr))
    return ok, orr


def reduce_by_key(keys, rids, rows, layout):
    k = _u64a(keys); r = _u32a(rids); rw = _rows_np(rows)
    n = k.shape[0]
    gk = np.empty(max(n, 1), np.uint64); gc = np.empty_like(gk); gs = np.empty_like(gk)
    gm = np.empty_like(gk); ng = np.zeros(1, np.uint64)
    _ck(lib().orc_reduce_by_key(k, r, n, _ptr(rw), layout.row_bytes, layout.val_off, layout.val_w,
                                gk, gc, gs, gm, ng))
    g = int(ng[0])
    return gk[:g], gc[:g], gs[:g], gm[:g]


def topk_by_sum(gkey, gsum, k=10):
    gk = _u64a(gkey); gs = _u64a(gsum)
    ok = np.empty(max(k, 1), np.uint64); osum = np.empty_like(ok); got = C.c_uint32(0)
    _ck(lib().orc_topk_by_sum(gk, gs, gk.shape[0], k, ok, osum, C.byref(got)))
    return ok[:got.value], osum[:got.value]


def median_by_key(keys, rids, rows, layout):
    k = _u64a(keys); r = _u32a(rids); rw = _rows_np(rows)
    n = k.shape[0]
    gk = np.empty(max(n, 1), np.uint64); gm = np.empty_like(gk); ng = np.zeros(1, np.uint64)
    _ck(lib().orc_median_by_key(k, r, n, _ptr(rw), layout.row_bytes, layout.val_off,
                                layout.val_w, gk, gm, ng))
    g = int(ng[0])
    return gk[:g], gm[:g]


def join(lk, lr, rk, rr, rows_l, rows_r, layout, pairs_cap=0):
    lk = _u64a(lk); lr = _u32a(lr); rk = _u64a(rk); rr = _u32a(rr)
    rl = _rows_np(rows_l); rrw = _rows_np(rows_r)
    cnt = np.zeros(1, np.uint64); sp = np.zeros(1, np.uint64); npairs = np.zeros(1, np.uint64)
    pairs = np.zeros((max(pairs_cap, 1), 3), np.uint64)
    _ck(lib().orc_join(lk, lr, lk.shape[0], rk, rr, rk.shape[0], _ptr(rl), _ptr(rrw),
                       layout.row_bytes, layout.val_off, layout.val_w, cnt, sp,
                       _ptr(pairs) if pairs_cap > 0 else None, pairs_cap, npairs))
    got = min(int(npairs[0]), pairs_cap)
    return int(cnt[0]), int(sp[0]), pairs[:got], int(npairs[0])


def materialize(rids, rows, layout):
    r = _u32a(rids); rw = _rows_np(rows)
    out = np.empty(r.shape[0] * layout.row_bytes, np.uint8)
    _ck(lib().orc_materialize(r, r.shape[0], _ptr(rw), layout.row_bytes, _ptr(out)))
    return out


def pwl_fit(sorted_keys, n_seg=1024):
    k = _u64a(sorted_keys)
    kmin = np.zeros(1, np.uint64); kmax = np.zeros(1, np.uint64)
    knots = np.empty(n_seg + 1, np.float32)
    _ck(lib().orc_pwl_fit(k, k.shape[0], n_seg, kmin, kmax, knots))
    return int(kmin[0]), int(kmax[0]), knots


def window_aggregate(rows, layout, win_len, n_win, k=10, n_threads=1, origin=0):
    r = _rows_np(rows)
    n = r.nbytes // layout.row_bytes
    g = np.zeros(n_win, np.uint64); tk = np.zeros(n_win * k, np.uint64)
    ts = np.zeros(n_win * k, np.uint64); cs = np.zeros(1, np.uint64)
    _ck(lib().orc_window_aggregate(_ptr(r), n, layout.row_bytes, layout.key_off, layout.val_off,
                                   layout.val_w, layout.ts_off, layout.ts_w, win_len, origin,
                                   n_win, k, n_threads, g, tk, ts, cs))
    return g, tk.reshape(n_win, k), ts.reshape(n_win, k), int(cs[0])
