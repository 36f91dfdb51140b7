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
        L.orc_topk_per_key.argtypes = [_u64p, _u32p, _u64, _vp, _i, _i, _i, _u32, _u64p, _u64p,
                                       _u32p, _u64p, _u64p]
        L.orc_unique_count_by_key.argtypes = [_u64p, _u32p, _u64, _vp, _i, _i, _i, _u64p, _u64p,
                                              _u64p]
        L.orc_reduce_all_windows.argtypes = [_vp, _u64, _i, _i, _i, _i, _i, _u64, _u64, _u32,
                                             _u64p, _u64p, _u64p, _u64p, _u64p]
        L.orc_select.argtypes = [_u64p, _u32p, _u64p, _u32, _vp, _i, _i, _i, _i, _i, _u64p, _u64p,
                                 _u64p, _u64p, _u32p, _u64p]
        L.orc_window_filter.argtypes = [_vp, _u64, _vp, _u64, _i, _i, _i, _i, _i, _i, _u64, _u64,
                                        _u32, _u64, _u64p, _u32p, _u64p]
        L.orc_keyswap.argtypes = [_u32p, _u64, _vp, _i, _i, _i, _u64p]
        L.orc_key_update.argtypes = [_u64p, _u64, _u64p, _u64p, _u64, _u64p]
        L.orc_key_writeback.argtypes = [_u64p, _u32p, _u64, _vp, _i, _i]
        L.orc_materialize_extract.argtypes = [_u32p, _u64, _vp, _i, _i, _u64, _vp, _u64p, _u32p]
        L.orc_sliding_aggregate.argtypes = [_vp, _u64, _i, _i, _i, _i, _i, _i, _u64, _u64, _u64,
                                            _u32, _u64, _u64p, _u64p, _u64p, _u64p, _u64p]
        L.orc_sort_rows_windowed.argtypes = [_vp, _u64, _i, _i, _i, _i, _u64, _u64, _u32, _vp,
                                             _u64p, _u64p]
        for f in ("orc_sort_rows_windowed", "orc_partition", "orc_extract", "orc_sort", "orc_sort_segmented", "orc_merge",
                  "orc_reduce_by_key", "orc_topk_by_sum", "orc_median_by_key", "orc_join",
                  "orc_materialize", "orc_pwl_fit", "orc_window_aggregate", "orc_topk_per_key",
                  "orc_unique_count_by_key", "orc_reduce_all_windows", "orc_select",
                  "orc_window_filter", "orc_keyswap", "orc_key_update", "orc_key_writeback",
                  "orc_materialize_extract", "orc_sliding_aggregate"):
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
    if isinstance(x, (list, tuple)):
        # Python ints at or above 2^63 would become float64 under np.asarray
        return np.array([int(v) for v in x], dtype=np.uint64)
    x = np.asarray(x)
    if x.dtype == np.int64:
        x = x.view(np.uint64)
    if x.dtype.kind == "f":
        raise TypeError("u64 arrays must be integers (floats would round)")
    return np.ascontiguousarray(x, dtype=np.uint64)


def _u32a(x):
    if hasattr(x, "detach"):
        x = x.detach().cpu().numpy()
    if isinstance(x, (list, tuple)):
        return np.array([int(v) for v in x], dtype=np.uint32)
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


def topk_per_key(keys, rids, rows, layout, k):
    """(gkey, gcnt, tn, topv[G, k]) in ascending key order; row g of topv holds
    the key's tn[g] largest values, descending, then zeros."""
    kk = _u64a(keys); r = _u32a(rids); rw = _rows_np(rows)
    n = kk.shape[0]
    gk = np.empty(max(n, 1), np.uint64); gc = np.empty_like(gk)
    tn = np.empty(max(n, 1), np.uint32); tv = np.empty(max(n, 1) * k, np.uint64)
    ng = np.zeros(1, np.uint64)
    _ck(lib().orc_topk_per_key(kk, r, n, _ptr(rw), layout.row_bytes, layout.val_off,
                               layout.val_w, k, gk, gc, tn, tv, ng))
    g = int(ng[0])
    return gk[:g], gc[:g], tn[:g], tv[:g * k].reshape(g, k)


def unique_count_by_key(keys, rids, rows, layout):
    kk = _u64a(keys); r = _u32a(rids); rw = _rows_np(rows)
    n = kk.shape[0]
    gk = np.empty(max(n, 1), np.uint64); gu = np.empty_like(gk); ng = np.zeros(1, np.uint64)
    _ck(lib().orc_unique_count_by_key(kk, r, n, _ptr(rw), layout.row_bytes, layout.val_off,
                                      layout.val_w, gk, gu, ng))
    g = int(ng[0])
    return gk[:g], gu[:g]


def reduce_all_windows(rows, layout, win_len, n_win, origin=0):
    """Per window: (count, sum_lo, sum_hi, max) arrays and the out-of-range count."""
    r = _rows_np(rows)
    n = r.nbytes // layout.row_bytes
    c = np.zeros(n_win, np.uint64); lo = np.zeros_like(c); hi = np.zeros_like(c)
    mx = np.zeros_like(c); oob = np.zeros(1, np.uint64)
    _ck(lib().orc_reduce_all_windows(_ptr(r), n, layout.row_bytes, layout.val_off, layout.val_w,
                                     layout.ts_off, layout.ts_w, win_len, origin, n_win, c, lo,
                                     hi, mx, oob))
    return c, lo, hi, mx, int(oob[0])


SELECT_OPS = {">": 0, ">=": 1, "<": 2, "<=": 3, "==": 4, "!=": 5}


def select(keys, rids, seg_off, num_lo, num_hi, den, op=">", column=0, rows=None, layout=None):
    """Survivors (keys, rids, seg_off) of x * den[s] <op> num[s] per segment."""
    kk = _u64a(keys); r = _u32a(rids); so = _u64a(seg_off)
    n_seg = so.shape[0] - 1
    lo = _u64a(num_lo); hi = _u64a(num_hi); dn = _u64a(den)
    ok = np.empty(max(kk.shape[0], 1), np.uint64); orr = np.empty(max(kk.shape[0], 1), np.uint32)
    oo = np.empty(n_seg + 1, np.uint64)
    rw = _rows_np(rows) if rows is not None else np.zeros(8, np.uint8)
    rb = layout.row_bytes if layout is not None else 8
    vo = layout.val_off if layout is not None else 0
    vw = layout.val_w if layout is not None else 8
    _ck(lib().orc_select(kk, r, so, n_seg, _ptr(rw), rb, vo, vw, column, SELECT_OPS[op], lo, hi,
                         dn, ok, orr, oo))
    m = int(oo[-1])
    return ok[:m], orr[:m], oo


def window_filter(rows_a, rows_b, layout, win_len, n_win, origin=0, rid_base_b=0):
    ra = _rows_np(rows_a); rb = _rows_np(rows_b)
    na = ra.nbytes // layout.row_bytes; nb = rb.nbytes // layout.row_bytes
    ok = np.empty(max(nb, 1), np.uint64); orr = np.empty(max(nb, 1), np.uint32)
    oo = np.empty(n_win + 1, np.uint64)
    _ck(lib().orc_window_filter(_ptr(ra), na, _ptr(rb), nb, layout.row_bytes, layout.key_off,
                                layout.val_off, layout.val_w, layout.ts_off, layout.ts_w, win_len,
                                origin, n_win, rid_base_b, ok, orr, oo))
    m = int(oo[-1])
    return ok[:m], orr[:m], oo


def keyswap(rids, rows, row_bytes, col_off, col_w):
    r = _u32a(rids); rw = _rows_np(rows)
    out = np.empty(max(r.shape[0], 1), np.uint64)
    _ck(lib().orc_keyswap(r, r.shape[0], _ptr(rw), row_bytes, col_off, col_w, out))
    return out[:r.shape[0]]


def key_update(keys, tkeys, tvals):
    """(updated copy of keys, number of keys missing from the table)."""
    kk = _u64a(keys).copy(); tk = _u64a(tkeys); tv = _u64a(tvals)
    miss = np.zeros(1, np.uint64)
    _ck(lib().orc_key_update(kk, kk.shape[0], tk, tv, tk.shape[0], miss))
    return kk, int(miss[0])


def key_writeback(keys, rids, rows, row_bytes, col_off):
    """A copy of the rows (bytes) with keys written to column col_off of their rows."""
    kk = _u64a(keys); r = _u32a(rids)
    out = np.array(_rows_np(rows), copy=True).view(np.uint8).reshape(-1)
    _ck(lib().orc_key_writeback(kk, r, kk.shape[0], _ptr(out), row_bytes, col_off))
    return out


def materialize_extract(rids, rows, row_bytes, key_off, rid_base=0):
    r = _u32a(rids); rw = _rows_np(rows)
    n = r.shape[0]
    out = np.empty(max(n, 1) * row_bytes, np.uint8)
    ok = np.empty(max(n, 1), np.uint64); orr = np.empty(max(n, 1), np.uint32)
    _ck(lib().orc_materialize_extract(r, n, _ptr(rw), row_bytes, key_off, rid_base, _ptr(out),
                                      ok, orr))
    return out[:n * row_bytes], ok[:n], orr[:n]


def sliding_aggregate(rows, layout, win_len, slide, n_win, origin=0, cap=None):
    """Per sliding window: (gkey, cnt, sum, max, gseg_off)."""
    r = _rows_np(rows)
    n = r.nbytes // layout.row_bytes
    cap = max(1, n * ((win_len + slide - 1) // slide + 1)) if cap is None else cap
    gk = np.empty(cap, np.uint64); gc = np.empty_like(gk); gs = np.empty_like(gk)
    gm = np.empty_like(gk); go = np.empty(n_win + 1, np.uint64)
    _ck(lib().orc_sliding_aggregate(_ptr(r), n, layout.row_bytes, layout.key_off, layout.val_off,
                                    layout.val_w, layout.ts_off, layout.ts_w, win_len, slide,
                                    origin, n_win, cap, gk, gc, gs, gm, go))
    g = int(go[-1])
    return gk[:g], gc[:g], gs[:g], gm[:g], go


def sort_rows_windowed(rows, layout, win_len, n_win, origin=0):
    """(rows ordered by (window, key) stably as bytes, win_off[n_win+1], oob)."""
    r = _rows_np(rows)
    n = r.nbytes // layout.row_bytes
    out = np.empty(max(n, 1) * layout.row_bytes, np.uint8)
    off = np.empty(n_win + 1, np.uint64); oob = np.zeros(1, np.uint64)
    _ck(lib().orc_sort_rows_windowed(_ptr(r), n, layout.row_bytes, layout.key_off, layout.ts_off,
                                     layout.ts_w, win_len, origin, n_win, _ptr(out), off, oob))
    return out[:n * layout.row_bytes], off, int(oob[0])
