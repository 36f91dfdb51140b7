"""ctypes binding of libkpa.so: the C-ABI calls under the same names.

Arguments are torch tensors on the current HIP device (PyTorch provides only
device memory and streams here).  Each function checks dtypes and shapes,
allocates the workspace the call asks for when none is given, and passes raw
pointers and the current stream.  Every step runs in the library's kernels;
there is no fallback: if libkpa.so is missing the import fails.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkpa.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python {_HERE}/build.py` "
                      "(or __graft_entry__.build())")

_lib = C.CDLL(LIB_PATH)

KPA_OK = 0
KPA_EINVAL = -1
KPA_EWORKSPACE = -2
KPA_ECAPACITY = -3
KPA_EBUDGET = -4
KPA_EUNSUPPORTED = -5
KPA_EHIP = -6
KPA_ETIMEOUT = -7
KPA_SORT_RADIX = 0
KPA_SORT_LEARNED = 1
KPA_Q_SUM = 0
KPA_Q_MEDIAN = 1
KPA_Q_JOIN = 2
KPA_PWL_MAX_SEG = 1024
KPA_MLP_PARAMS = 1153
PWL_MODEL_BYTES = 8 + 8 + 4 + 4 + 4 * (KPA_PWL_MAX_SEG + 1) + 12  # sizeof(kpa_pwl_model)
SORT_STATS_WORDS = 7
KPA_SEL_KEY = 0
KPA_SEL_VALUE = 1
SELECT_OPS = {">": 0, ">=": 1, "<": 2, "<=": 3, "==": 4, "!=": 5}


class KpaError(RuntimeError):
    def __init__(self, fn, code):
        msg = _lib.kpa_last_error_string().decode(errors="replace")
        super().__init__(f"{fn} failed with status {code}: {msg}")
        self.code = code


class kpa_batch_config(C.Structure):
    _fields_ = [("small_cap", C.c_uint32), ("mid_cap", C.c_uint32), ("grid", C.c_uint32),
                ("large_algo", C.c_uint32), ("bucket_log2", C.c_uint32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class kpa_server_config(C.Structure):
    _fields_ = [("budget_bytes", C.c_uint64), ("slots", C.c_uint32), ("rows_in_host", C.c_uint32),
                ("max_bundle_rows", C.c_uint64), ("max_row_bytes", C.c_uint32),
                ("max_pending", C.c_uint32), ("reserve_pct", C.c_uint32),
                ("max_live_bundles", C.c_uint32), ("host_pool_bytes", C.c_uint64),
                ("placement", C.c_uint32), ("monitor_ms", C.c_uint32),
                ("target_delay_ms", C.c_double), ("host_bw_gbs", C.c_double),
                ("keep_groups", C.c_uint32), ("seed", C.c_uint32)]


KPA_PLACE_DEVICE = 0
KPA_PLACE_BALANCED = 1
KPA_PLACE_HOST = 2


class kpa_monitor_sample(C.Structure):
    _fields_ = [("t_s", C.c_double), ("hbm_util", C.c_double), ("bw_util", C.c_double),
                ("k_low", C.c_double), ("k_high", C.c_double), ("delay_ms", C.c_double),
                ("hbm_bytes", C.c_uint64), ("host_bytes", C.c_uint64), ("waits", C.c_uint64),
                ("bundles_host", C.c_uint64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class kpa_window_result(C.Structure):
    _fields_ = [("query", C.c_uint32), ("kind", C.c_uint32), ("window", C.c_uint64),
                ("rows", C.c_uint64 * 2), ("groups", C.c_uint64), ("total", C.c_uint64),
                ("digest", C.c_uint64), ("n_top", C.c_uint32), ("reserved", C.c_uint32),
                ("top_key", C.c_uint64 * 10), ("top_sum", C.c_uint64 * 10),
                ("latency_ms", C.c_double), ("groups_data", C.POINTER(C.c_uint64)),
                ("groups_words", C.c_uint64), ("runs", C.c_uint32), ("runs_host", C.c_uint32)]

    def as_dict(self):
        return {"query": self.query, "kind": self.kind, "window": self.window,
                "rows": (self.rows[0], self.rows[1]), "groups": self.groups, "total": self.total,
                "digest": self.digest, "top_key": list(self.top_key)[:self.n_top],
                "top_sum": list(self.top_sum)[:self.n_top], "latency_ms": self.latency_ms,
                "runs": self.runs, "runs_host": self.runs_host}


class kpa_server_statistics(C.Structure):
    _fields_ = [("bundles", C.c_uint64), ("rows", C.c_uint64), ("late_rows", C.c_uint64),
                ("windows_closed", C.c_uint64), ("backpressure_waits", C.c_uint64),
                ("pool_peak_bytes", C.c_uint64), ("pool_bytes", C.c_uint64),
                ("p50_ms", C.c_double), ("p99_ms", C.c_double), ("max_ms", C.c_double),
                ("elapsed_s", C.c_double), ("mrec_per_s", C.c_double),
                ("bundles_on_host", C.c_uint64), ("host_pool_bytes", C.c_uint64),
                ("host_pool_peak_bytes", C.c_uint64), ("k_low", C.c_double),
                ("k_high", C.c_double), ("host_bw_gbs", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class kpa_row_layout(C.Structure):
    _fields_ = [("row_bytes", C.c_uint32), ("key_off", C.c_uint32), ("val_off", C.c_uint32),
                ("val_w", C.c_uint32), ("ts_off", C.c_uint32), ("ts_w", C.c_uint32)]


_vp = C.c_void_p
_u64 = C.c_uint64
_u32 = C.c_uint32
_f32 = C.c_float
_sz = C.POINTER(C.c_size_t)
_lay = C.POINTER(kpa_row_layout)

_SIGS = {
    "kpa_version": ([], C.c_int32),
    "kpa_last_error_string": ([], C.c_char_p),
    "kpa_last_hip_error": ([], C.c_int32),
    "kpa_device_check": ([C.POINTER(C.c_int32)], C.c_int32),
    "kpa_profile_enable": ([C.c_int32], C.c_int32),
    "kpa_profile_collect": ([], C.c_int32),
    "kpa_profile_get": ([C.c_char_p, C.POINTER(_u64), C.POINTER(C.c_double)], C.c_int32),
    "kpa_profile_names": ([C.c_char_p, C.c_size_t], C.c_int32),
    "kpa_extract": ([_vp, _u64, _lay, _u32, _vp, _vp, _vp, _vp], C.c_int32),
    "kpa_partition_windows_workspace_size": ([_u64, _u32, _sz], C.c_int32),
    "kpa_partition_windows": ([_vp, _u64, _lay, _u64, _u64, _u32, _u32, _vp, _vp, _vp, _vp, _vp,
                               _vp, C.c_size_t, _vp], C.c_int32),
    "kpa_sort_workspace_size": ([_u64, _u32, C.c_int, _sz], C.c_int32),
    "kpa_sort_segmented": ([_vp, _vp, _vp, _vp, _vp, _u32, _u64, C.c_int, _vp, _vp, _vp,
                            C.c_size_t, _vp], C.c_int32),
    "kpa_sort": ([_vp, _vp, _u64, _vp, _vp, C.c_int, _vp, _vp, _vp, C.c_size_t, _vp], C.c_int32),
    "kpa_sort_vals_workspace_size": ([_u64, _u32, C.c_int, _sz], C.c_int32),
    "kpa_sort_segmented_vals": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp, _u32, _u64, C.c_int, _vp,
                                 _vp, _vp, C.c_size_t, _vp], C.c_int32),
    "kpa_batch_config_default": ([C.c_int, C.POINTER(kpa_batch_config)], C.c_int32),
    "kpa_batch_sort_workspace_size": ([_u64, _u32, C.POINTER(kpa_batch_config), _sz], C.c_int32),
    "kpa_batch_sort": ([_vp, _vp, _vp, _vp, _vp, _u32, _u64, C.POINTER(kpa_batch_config), _vp,
                        _vp, _vp, C.c_size_t, _vp], C.c_int32),
    "kpa_batch_sort_vals_workspace_size": ([_u64, _u32, C.POINTER(kpa_batch_config), _sz],
                                           C.c_int32),
    "kpa_batch_sort_vals": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp, _u32, _u64,
                             C.POINTER(kpa_batch_config), _vp, _vp, _vp, C.c_size_t, _vp],
                            C.c_int32),
    "kpa_batch_autotune": ([_vp, _vp, _vp, _vp, _vp, _u32, _u64, C.c_int, _vp, _vp, C.c_size_t,
                            _u32, C.c_char_p, C.POINTER(kpa_batch_config), C.POINTER(_f32), _vp],
                           C.c_int32),
    "kpa_graph_begin": ([_vp], C.c_int32),
    "kpa_graph_end": ([_vp, C.POINTER(_vp)], C.c_int32),
    "kpa_graph_launch": ([_vp, _vp], C.c_int32),
    "kpa_graph_destroy": ([_vp], C.c_int32),
    "kpa_ingest_bundle": ([_vp, _u64, _lay, _u64, _vp, _vp], C.c_int32),
    "kpa_server_config_default": ([C.POINTER(kpa_server_config)], C.c_int32),
    "kpa_server_create": ([C.POINTER(kpa_server_config), C.POINTER(_vp)], C.c_int32),
    "kpa_server_add_query": ([_vp, C.c_int, _lay, _u64, _u64, C.POINTER(_u32)], C.c_int32),
    "kpa_server_submit": ([_vp, _u32, _u32, _vp, _u64, _u64, _u64, _u64, C.c_int32], C.c_int32),
    "kpa_server_watermark": ([_vp, _u32, _u64], C.c_int32),
    "kpa_server_poll": ([_vp, C.POINTER(kpa_window_result), C.POINTER(C.c_int32), C.c_int32],
                        C.c_int32),
    "kpa_server_drain": ([_vp, C.c_int32], C.c_int32),
    "kpa_server_stats": ([_vp, C.POINTER(kpa_server_statistics)], C.c_int32),
    "kpa_server_destroy": ([_vp], C.c_int32),
    "kpa_server_release_groups": ([_vp, C.POINTER(C.c_uint64)], C.c_int32),
    "kpa_server_trace": ([_vp, C.POINTER(kpa_monitor_sample), _u32, C.POINTER(_u32)], C.c_int32),
    "kpa_balance_knob_update": ([C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_double,
                                 C.c_double, C.c_double, C.c_double], C.c_int32),
    "kpa_merge_workspace_size": ([_u64, _u64, _sz], C.c_int32),
    "kpa_merge": ([_vp, _vp, _u64, _vp, _vp, _u64, _vp, _vp, _vp, C.c_size_t, _vp], C.c_int32),
    "kpa_merge_runs_workspace_size": ([_u64, _sz], C.c_int32),
    "kpa_merge_runs": ([_vp, _vp, C.POINTER(_u64), _u32, _vp, _vp, _vp, C.c_size_t, _vp],
                       C.c_int32),
    "kpa_reduce_by_key_workspace_size": ([_u64, _u32, _sz], C.c_int32),
    "kpa_reduce_by_key": ([_vp, _vp, _vp, _u32, _u64, _vp, _lay, _vp, _vp, _vp, _vp, _vp, _vp,
                           _vp, C.c_size_t, _vp], C.c_int32),
    "kpa_reduce_by_key_noalloc": ([_vp, _vp, _vp, _u32, _u64, _vp, _lay, _vp, _vp, _vp, _vp,
                                   _vp, _vp, _vp], C.c_int32),
    "kpa_topk_by_sum_workspace_size": ([_u64, _u32, _sz], C.c_int32),
    "kpa_topk_by_sum": ([_vp, _vp, _vp, _u32, _u64, _u32, _vp, _vp, _vp, _vp, C.c_size_t, _vp],
                        C.c_int32),
    "kpa_median_by_key_workspace_size": ([_u64, _u32, _sz], C.c_int32),
    "kpa_median_by_key": ([_vp, _vp, _vp, _u32, _u64, _vp, _lay, _vp, _vp, _vp, _vp, _vp, _vp,
                           C.c_size_t, _vp], C.c_int32),
    "kpa_join_workspace_size": ([_u64, _u64, _u32, _sz], C.c_int32),
    "kpa_join_runs_workspace_size": ([_u64, _u64, _u32, _sz], C.c_int32),
    "kpa_join_runs": ([_vp, _vp, _vp, _vp, _u64, _vp, _vp, _vp, _vp, _u64, _u32, _vp, _vp, _vp,
                       C.c_size_t, _vp], C.c_int32),
    "kpa_join": ([_vp, _vp, _vp, _u64, _vp, _vp, _vp, _u64, _u32, _vp, _vp, _lay, _vp, _vp, _vp,
                  _u64, _vp, _vp, C.c_size_t, _vp], C.c_int32),
    "kpa_materialize": ([_vp, _u64, _vp, _u32, _vp, _vp], C.c_int32),
    "kpa_materialize_extract": ([_vp, _u64, _vp, _u32, _u32, _u32, _vp, _vp, _vp, _vp], C.c_int32),
    "kpa_keyswap": ([_vp, _u64, _vp, _u32, _u32, _u32, _vp, _vp], C.c_int32),
    "kpa_key_update": ([_vp, _u64, _vp, _vp, _u64, _vp, _vp], C.c_int32),
    "kpa_key_writeback": ([_vp, _vp, _u64, _vp, _u32, _u32, _vp], C.c_int32),
    "kpa_select_workspace_size": ([_u64, _u32, _sz], C.c_int32),
    "kpa_select": ([_vp, _vp, _vp, _u32, _u64, _vp, _lay, C.c_int, C.c_int, _vp, _vp, _vp, _vp,
                    _vp, _vp, _vp, C.c_size_t, _vp], C.c_int32),
    "kpa_reduce_all_windows_workspace_size": ([_u32, _sz], C.c_int32),
    "kpa_reduce_all_windows": ([_vp, _u64, _lay, _u64, _u64, _u32, _vp, _vp, _vp, _vp, _vp, _vp,
                                C.c_size_t, _vp], C.c_int32),
    "kpa_run_stats_workspace_size": ([_u64, _u32, _sz], C.c_int32),
    "kpa_topk_per_key": ([_vp, _vp, _vp, _u32, _u64, _vp, _lay, _u32, _vp, _vp, _vp, _vp, _vp,
                          _vp, C.c_size_t, _vp], C.c_int32),
    "kpa_unique_count_by_key": ([_vp, _vp, _vp, _u32, _u64, _vp, _lay, _vp, _vp, _vp, _vp,
                                 C.c_size_t, _vp], C.c_int32),
    "kpa_sort_rows_windowed_workspace_size": ([_u64, _u32, _sz], C.c_int32),
    "kpa_sort_rows_windowed": ([_vp, _u64, _lay, _u64, _u64, _u32, _vp, _vp, _vp, _vp, C.c_size_t,
                                _vp], C.c_int32),
    "kpa_hash_groupby_workspace_size": ([_u64, _sz], C.c_int32),
    "kpa_hash_groupby": ([_vp, _u64, _lay, _u64, _vp, _vp, _vp, _vp, _u64, _vp, _vp, C.c_size_t,
                          _vp], C.c_int32),
    "kpa_window_panes": ([_vp, _vp, _u32, _u32, _vp, _vp, _vp, _u64, _vp], C.c_int32),
    "kpa_partition_kpa": ([_vp, _vp, _u64, _u64, _u64, _u32, _vp, _vp, _vp, _vp, _vp, C.c_size_t,
                           _vp], C.c_int32),
    "kpa_pwl_fit": ([_vp, _vp, _u32, _u32, _vp, _vp], C.c_int32),
    "kpa_mlp_training_set": ([_vp, _u64, _u32, _vp, _vp, _vp, _vp], C.c_int32),
    "kpa_mlp_forward": ([_vp, _vp, _u32, _vp, _vp], C.c_int32),
    "kpa_mlp_loss_grad_workspace_size": ([_u32, _sz], C.c_int32),
    "kpa_mlp_loss_grad": ([_vp, _vp, _vp, _u32, _vp, _vp, _vp, C.c_size_t, _vp], C.c_int32),
    "kpa_mlp_adam_step": ([_vp, _vp, _vp, _vp, _u32, _f32, _f32, _f32, _f32, _vp], C.c_int32),
    "kpa_mlp_train": ([_vp, _vp, _vp, _vp, _vp, _u32, _u32, _u32, _f32, _vp, _vp, C.c_size_t,
                       _vp], C.c_int32),
    "kpa_mlp_to_pwl": ([_vp, _u32, _vp, _vp], C.c_int32),
    "kpa_mlp_init": ([_vp, _vp, _vp], C.c_int32),
}

EXPORTED = []
for _name, (_args, _res) in _SIGS.items():
    if hasattr(_lib, _name):
        _f = getattr(_lib, _name)
        _f.argtypes = _args
        _f.restype = _res
        EXPORTED.append(_name)


def _call(name, *args):
    rc = getattr(_lib, name)(*args)
    if rc != KPA_OK:
        raise KpaError(name, rc)


def _p(t):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ws_size(fn, *args):
    n = C.c_size_t(0)
    _call(fn, *args, C.byref(n))
    return int(n.value)


def _ws(nbytes, device, ws=None, stream=None):
    """The caller's workspace, or a new one; a new one is marked as used on
    `stream`, so that the caching allocator does not hand it out again
    before the work enqueued there has finished with it."""
    if ws is not None:
        if ws.numel() * ws.element_size() < nbytes:
            raise ValueError(f"workspace of {ws.numel()} bytes < {nbytes}")
        return ws
    t = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
    if stream is not None:
        t.record_stream(stream)
    return t


def _check(t, dtype, name):
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def layout_struct(layout):
    return kpa_row_layout(layout.row_bytes, layout.key_off, layout.val_off, layout.val_w,
                          layout.ts_off, layout.ts_w)


def rows_count(rows, layout):
    return rows.numel() * rows.element_size() // layout.row_bytes


# ------------------------------------------------------------------ calls --

def kpa_version():
    return int(_lib.kpa_version())


def kpa_device_check():
    v = C.c_int32(0)
    _call("kpa_device_check", C.byref(v))
    return bool(v.value)


def kpa_profile_enable(on=True):
    _call("kpa_profile_enable", 1 if on else 0)


def kpa_profile_collect():
    _call("kpa_profile_collect")


def kpa_profile_get(name):
    """(launches, total milliseconds) of one kernel since the last enable."""
    n = C.c_uint64(0)
    ms = C.c_double(0.0)
    _call("kpa_profile_get", name.encode(), C.byref(n), C.byref(ms))
    return int(n.value), float(ms.value)


def kpa_profile_names():
    buf = C.create_string_buffer(4096)
    _call("kpa_profile_names", buf, 4096)
    v = buf.value.decode()
    return [x for x in v.split(",") if x]


def kpa_extract(rows, layout, rid_base=0, out_keys=None, out_rids=None, stream=None,
                out_vals=None, n=None, with_rids=True):
    """Returns (keys, rids); out_vals (n int64), when given, also receives the
    value column.  with_rids=False: no row ids are written (rids is None)."""
    n = rows_count(rows, layout) if n is None else n
    dev = rows.device
    out_keys = torch.empty(n, dtype=torch.int64, device=dev) if out_keys is None else out_keys
    if not with_rids:
        out_rids = None
    elif out_rids is None:
        out_rids = torch.empty(n, dtype=torch.int32, device=dev)
    L = layout_struct(layout)
    _call("kpa_extract", _p(rows), n, C.byref(L), rid_base, _p(out_keys), _p(out_rids),
          _p(out_vals), _stream(stream))
    return out_keys, out_rids


def kpa_partition_windows(rows, layout, win_len, n_win, win_origin=0, rid_base=0, n=None,
                          out_keys=None, out_rids=None, out_win_off=None, out_oob=None, ws=None,
                          stream=None, out_vals=None):
    """Returns (keys, rids, win_off, oob).  out_vals, when given (n int64), also
    receives the value column of every row in arrival order."""
    n = rows_count(rows, layout) if n is None else n
    dev = rows.device
    out_keys = torch.empty(max(n, 1), dtype=torch.int64, device=dev) if out_keys is None else out_keys
    out_rids = torch.empty(max(n, 1), dtype=torch.int32, device=dev) if out_rids is None else out_rids
    out_win_off = (torch.empty(n_win + 1, dtype=torch.int64, device=dev)
                   if out_win_off is None else out_win_off)
    out_oob = torch.empty(1, dtype=torch.int64, device=dev) if out_oob is None else out_oob
    nb = _ws_size("kpa_partition_windows_workspace_size", n, n_win)
    ws = _ws(nb, dev, ws, stream)
    L = layout_struct(layout)
    _call("kpa_partition_windows", _p(rows), n, C.byref(L), win_len, win_origin, n_win, rid_base,
          _p(out_keys), _p(out_rids), _p(out_vals), _p(out_win_off), _p(out_oob), _p(ws),
          ws.numel() * ws.element_size(), _stream(stream))
    return out_keys, out_rids, out_win_off, out_oob


def kpa_sort_workspace_size(n_cap, n_seg=1, algo=KPA_SORT_RADIX):
    return _ws_size("kpa_sort_workspace_size", n_cap, n_seg, algo)


def kpa_sort_segmented(keys_in, rids_in, seg_off, n_cap=None, algo=KPA_SORT_RADIX, models=None,
                       stats=None, keys_out=None, rids_out=None, ws=None, stream=None):
    _check(keys_in, torch.int64, "keys_in")
    if rids_in is not None:   # None: row ids are the entries' positions
        _check(rids_in, torch.int32, "rids_in")
    n_seg = seg_off.numel() - 1
    n_cap = keys_in.numel() if n_cap is None else n_cap
    dev = keys_in.device
    keys_out = torch.empty_like(keys_in) if keys_out is None else keys_out
    rids_out = (torch.empty(keys_in.numel(), dtype=torch.int32, device=dev)
                if rids_out is None else rids_out)
    nb = kpa_sort_workspace_size(n_cap, n_seg, algo)
    ws = _ws(nb, dev, ws, stream)
    _call("kpa_sort_segmented", _p(keys_in), _p(rids_in), _p(keys_out), _p(rids_out), _p(seg_off),
          n_seg, n_cap, algo, _p(models), _p(stats), _p(ws), ws.numel() * ws.element_size(),
          _stream(stream))
    return keys_out, rids_out


def kpa_sort_vals_workspace_size(n_cap, n_seg=1, algo=KPA_SORT_RADIX):
    return _ws_size("kpa_sort_vals_workspace_size", n_cap, n_seg, algo)


def kpa_sort_segmented_vals(keys_in, rids_in, vals_in, seg_off, n_cap=None, algo=KPA_SORT_RADIX,
                            models=None, stats=None, keys_out=None, rids_out=None, vals_out=None,
                            ws=None, stream=None):
    """kpa_sort_segmented with an 8-byte column carried beside the KPA;
    returns (keys_out, rids_out, vals_out)."""
    _check(keys_in, torch.int64, "keys_in")
    if rids_in is not None:   # None: row ids are the entries' positions
        _check(rids_in, torch.int32, "rids_in")
    _check(vals_in, torch.int64, "vals_in")
    n_seg = seg_off.numel() - 1
    n_cap = keys_in.numel() if n_cap is None else n_cap
    dev = keys_in.device
    keys_out = torch.empty_like(keys_in) if keys_out is None else keys_out
    rids_out = (torch.empty(keys_in.numel(), dtype=torch.int32, device=dev)
                if rids_out is None else rids_out)
    vals_out = torch.empty_like(vals_in) if vals_out is None else vals_out
    ws = _ws(kpa_sort_vals_workspace_size(n_cap, n_seg, algo), dev, ws, stream)
    _call("kpa_sort_segmented_vals", _p(keys_in), _p(rids_in), _p(vals_in), _p(keys_out),
          _p(rids_out), _p(vals_out), _p(seg_off), n_seg, n_cap, algo, _p(models), _p(stats),
          _p(ws), ws.numel() * ws.element_size(), _stream(stream))
    return keys_out, rids_out, vals_out


def kpa_sort(keys_in, rids_in, algo=KPA_SORT_RADIX, model=None, stats=None, keys_out=None,
             rids_out=None, ws=None, stream=None):
    _check(keys_in, torch.int64, "keys_in")
    _check(rids_in, torch.int32, "rids_in")
    n = keys_in.numel()
    dev = keys_in.device
    keys_out = torch.empty_like(keys_in) if keys_out is None else keys_out
    rids_out = torch.empty_like(rids_in) if rids_out is None else rids_out
    nb = kpa_sort_workspace_size(n, 1, algo)
    ws = _ws(nb, dev, ws, stream)
    _call("kpa_sort", _p(keys_in), _p(rids_in), n, _p(keys_out), _p(rids_out), algo, _p(model),
          _p(stats), _p(ws), ws.numel() * ws.element_size(), _stream(stream))
    return keys_out, rids_out


def kpa_batch_config_default(large_algo=KPA_SORT_RADIX):
    cfg = kpa_batch_config()
    _call("kpa_batch_config_default", large_algo, C.byref(cfg))
    return cfg


def batch_config(small_cap=4096, mid_cap=1 << 16, grid=0, large_algo=KPA_SORT_RADIX,
                 bucket_log2=0):
    return kpa_batch_config(small_cap, mid_cap, grid, large_algo, bucket_log2)


def kpa_batch_sort_workspace_size(n_cap, n_seg, cfg):
    return _ws_size("kpa_batch_sort_workspace_size", n_cap, n_seg, C.byref(cfg))


def kpa_batch_sort(keys_in, rids_in, seg_off, cfg=None, n_cap=None, models=None, stats=None,
                   keys_out=None, rids_out=None, ws=None, stream=None):
    _check(keys_in, torch.int64, "keys_in")
    if rids_in is not None:   # None: row ids are the entries' positions
        _check(rids_in, torch.int32, "rids_in")
    cfg = kpa_batch_config_default() if cfg is None else cfg
    n_seg = seg_off.numel() - 1
    n_cap = keys_in.numel() if n_cap is None else n_cap
    dev = keys_in.device
    keys_out = torch.empty_like(keys_in) if keys_out is None else keys_out
    rids_out = (torch.empty(keys_in.numel(), dtype=torch.int32, device=dev)
                if rids_out is None else rids_out)
    ws = _ws(kpa_batch_sort_workspace_size(n_cap, n_seg, cfg), dev, ws, stream)
    _call("kpa_batch_sort", _p(keys_in), _p(rids_in), _p(keys_out), _p(rids_out), _p(seg_off),
          n_seg, n_cap, C.byref(cfg), _p(models), _p(stats), _p(ws),
          ws.numel() * ws.element_size(), _stream(stream))
    return keys_out, rids_out


def kpa_batch_sort_vals_workspace_size(n_cap, n_seg, cfg):
    return _ws_size("kpa_batch_sort_vals_workspace_size", n_cap, n_seg, C.byref(cfg))


def kpa_batch_sort_vals(keys_in, rids_in, vals_in, seg_off, cfg=None, n_cap=None, models=None,
                        stats=None, keys_out=None, rids_out=None, vals_out=None, ws=None,
                        stream=None):
    """kpa_batch_sort with an 8-byte column carried beside the KPA; returns
    (keys_out, rids_out, vals_out)."""
    _check(keys_in, torch.int64, "keys_in")
    if rids_in is not None:   # None: row ids are the entries' positions
        _check(rids_in, torch.int32, "rids_in")
    _check(vals_in, torch.int64, "vals_in")
    cfg = kpa_batch_config_default() if cfg is None else cfg
    n_seg = seg_off.numel() - 1
    n_cap = keys_in.numel() if n_cap is None else n_cap
    dev = keys_in.device
    keys_out = torch.empty_like(keys_in) if keys_out is None else keys_out
    rids_out = (torch.empty(keys_in.numel(), dtype=torch.int32, device=dev)
                if rids_out is None else rids_out)
    vals_out = torch.empty_like(vals_in) if vals_out is None else vals_out
    ws = _ws(kpa_batch_sort_vals_workspace_size(n_cap, n_seg, cfg), dev, ws, stream)
    _call("kpa_batch_sort_vals", _p(keys_in), _p(rids_in), _p(vals_in), _p(keys_out),
          _p(rids_out), _p(vals_out), _p(seg_off), n_seg, n_cap, C.byref(cfg), _p(models),
          _p(stats), _p(ws), ws.numel() * ws.element_size(), _stream(stream))
    return keys_out, rids_out, vals_out


def kpa_batch_autotune(keys_in, rids_in, seg_off, large_algo=KPA_SORT_RADIX, n_cap=None,
                       models=None, reps=2, cache_path=None, keys_out=None, rids_out=None,
                       ws=None, stream=None):
    """Returns (best kpa_batch_config, its mean milliseconds)."""
    _check(keys_in, torch.int64, "keys_in")
    if rids_in is not None:   # None: row ids are the entries' positions
        _check(rids_in, torch.int32, "rids_in")
    n_seg = seg_off.numel() - 1
    n_cap = keys_in.numel() if n_cap is None else n_cap
    dev = keys_in.device
    keys_out = torch.empty_like(keys_in) if keys_out is None else keys_out
    rids_out = (torch.empty(keys_in.numel(), dtype=torch.int32, device=dev)
                if rids_out is None else rids_out)
    ws = _ws(kpa_batch_sort_workspace_size(n_cap, n_seg, kpa_batch_config_default(large_algo)),
             dev, ws, stream)
    best = kpa_batch_config()
    ms = C.c_float(0.0)
    _call("kpa_batch_autotune", _p(keys_in), _p(rids_in), _p(keys_out), _p(rids_out), _p(seg_off),
          n_seg, n_cap, large_algo, _p(models), _p(ws), ws.numel() * ws.element_size(), reps,
          None if cache_path is None else os.fsencode(cache_path), C.byref(best), C.byref(ms),
          _stream(stream))
    return best, float(ms.value)


class Graph:
    """A captured sequence of library calls (kpa_graph_*).  Use as
    ``with Graph.capture(stream) as g: ...calls on stream...`` then
    ``g.launch(stream)``.  Buffers used inside must outlive the graph."""

    def __init__(self):
        self.h = C.c_void_p(None)
        self._stream = None

    @classmethod
    def capture(cls, stream):
        g = cls()
        g._stream = stream
        return g

    def __enter__(self):
        _call("kpa_graph_begin", _stream(self._stream))
        return self

    def __exit__(self, et, ev, tb):
        h = C.c_void_p(None)
        rc = _lib.kpa_graph_end(_stream(self._stream), C.byref(h))
        self.h = h
        if et is None and rc != KPA_OK:
            raise KpaError("kpa_graph_end", rc)
        return False

    def launch(self, stream=None):
        _call("kpa_graph_launch", self.h, _stream(stream if stream is not None else self._stream))

    def destroy(self):
        if self.h:
            _call("kpa_graph_destroy", self.h)
            self.h = C.c_void_p(None)

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def kpa_graph_begin(stream):
    _call("kpa_graph_begin", _stream(stream))


def kpa_graph_end(stream):
    h = C.c_void_p(None)
    _call("kpa_graph_end", _stream(stream), C.byref(h))
    return h


def kpa_graph_launch(graph, stream=None):
    _call("kpa_graph_launch", graph, _stream(stream))


def kpa_graph_destroy(graph):
    _call("kpa_graph_destroy", graph)


def kpa_merge(a_keys, a_rids, b_keys, b_rids, out_keys=None, out_rids=None, ws=None, stream=None):
    na, nb_ = a_keys.numel(), b_keys.numel()
    dev = a_keys.device
    out_keys = torch.empty(na + nb_, dtype=torch.int64, device=dev) if out_keys is None else out_keys
    out_rids = torch.empty(na + nb_, dtype=torch.int32, device=dev) if out_rids is None else out_rids
    nb = _ws_size("kpa_merge_workspace_size", na, nb_)
    ws = _ws(nb, dev, ws, stream)
    _call("kpa_merge", _p(a_keys), _p(a_rids), na, _p(b_keys), _p(b_rids), nb_, _p(out_keys),
          _p(out_rids), _p(ws), ws.numel() * ws.element_size(), _stream(stream))
    return out_keys, out_rids


def kpa_merge_runs(keys, rids, run_off, out_keys=None, out_rids=None, ws=None, stream=None):
    """run_off: host list/array of n_runs+1 offsets.  keys/rids are clobbered."""
    n = keys.numel()
    dev = keys.device
    offs = (C.c_uint64 * len(run_off))(*[int(x) for x in run_off])
    out_keys = torch.empty_like(keys) if out_keys is None else out_keys
    out_rids = torch.empty_like(rids) if out_rids is None else out_rids
    nb = _ws_size("kpa_merge_runs_workspace_size", n)
    ws = _ws(nb, dev, ws, stream)
    _call("kpa_merge_runs", _p(keys), _p(rids), offs, len(run_off) - 1, _p(out_keys), _p(out_rids),
          _p(ws), ws.numel() * ws.element_size(), _stream(stream))
    return out_keys, out_rids


def kpa_reduce_by_key(keys, rids, seg_off, rows, layout, n_cap=None, want=("cnt", "sum", "max"),
                      ws=None, stream=None, outs=None):
    n_seg = seg_off.numel() - 1
    n_cap = keys.numel() if n_cap is None else n_cap
    dev = keys.device
    cap = max(n_cap, 1)
    o = outs or {}
    def get(name, size):   # allocate only what the caller did not pass
        return o[name] if name in o else torch.empty(size, dtype=torch.int64, device=dev)
    gkey = get("gkey", cap)
    outs_t = {w: get(w, cap) for w in want}
    gseg = get("gseg_off", n_seg + 1)
    nb = _ws_size("kpa_reduce_by_key_workspace_size", n_cap, n_seg)
    ws = _ws(nb, dev, ws, stream)
    L = layout_struct(layout) if layout is not None else None   # counts only: no rows
    _call("kpa_reduce_by_key", _p(keys), _p(rids), _p(seg_off), n_seg, n_cap, _p(rows),
          C.byref(L) if L is not None else None,
          _p(gkey), _p(outs_t.get("cnt")), _p(outs_t.get("sum")), _p(outs_t.get("max")),
          _p(outs_t.get("gstart")), _p(gseg), _p(ws), ws.numel() * ws.element_size(),
          _stream(stream))
    return gkey, outs_t, gseg


def kpa_reduce_by_key_noalloc(keys, rids, seg_off, rows, layout, outs, n_cap=None,
                              want=("cnt", "sum", "max"), stream=None):
    """kpa_reduce_by_key without a workspace (the library's static scratch);
    outs must hold every output tensor: gkey, gseg_off and the wanted ones."""
    n_seg = seg_off.numel() - 1
    n_cap = keys.numel() if n_cap is None else n_cap
    L = layout_struct(layout)
    _call("kpa_reduce_by_key_noalloc", _p(keys), _p(rids), _p(seg_off), n_seg, n_cap, _p(rows),
          C.byref(L), _p(outs["gkey"]), _p(outs.get("cnt") if "cnt" in want else None),
          _p(outs.get("sum") if "sum" in want else None),
          _p(outs.get("max") if "max" in want else None), _p(outs.get("gstart")),
          _p(outs["gseg_off"]), _stream(stream))
    return outs


def kpa_topk_by_sum(gkey, gsum, gseg_off, k=10, g_cap=None, ws=None, stream=None, outs=None):
    n_seg = gseg_off.numel() - 1
    g_cap = gkey.numel() if g_cap is None else g_cap
    dev = gkey.device
    o = outs or {}
    ok = o["key"] if "key" in o else torch.empty(n_seg * k, dtype=torch.int64, device=dev)
    osum = o["sum"] if "sum" in o else torch.empty(n_seg * k, dtype=torch.int64, device=dev)
    on = o["n"] if "n" in o else torch.empty(n_seg, dtype=torch.int32, device=dev)
    nb = _ws_size("kpa_topk_by_sum_workspace_size", g_cap, n_seg)
    ws = _ws(nb, dev, ws, stream)
    _call("kpa_topk_by_sum", _p(gkey), _p(gsum), _p(gseg_off), n_seg, g_cap, k, _p(ok), _p(osum),
          _p(on), _p(ws), ws.numel() * ws.element_size(), _stream(stream))
    return ok, osum, on


def kpa_median_by_key(keys, rids, seg_off, rows, layout, n_cap=None, ws=None, stream=None,
                      outs=None):
    """Returns (gkey, gmed, gseg_off); outs may also name "cnt" and "sum"
    arrays, which then receive each group's count and sum of values."""
    n_seg = seg_off.numel() - 1
    n_cap = keys.numel() if n_cap is None else n_cap
    dev = keys.device
    cap = max(n_cap, 1)
    o = outs or {}
    gkey = o["gkey"] if "gkey" in o else torch.empty(cap, dtype=torch.int64, device=dev)
    gmed = o["gmed"] if "gmed" in o else torch.empty(cap, dtype=torch.int64, device=dev)
    gseg = o["gseg_off"] if "gseg_off" in o else torch.empty(n_seg + 1, dtype=torch.int64,
                                                               device=dev)
    nb = _ws_size("kpa_median_by_key_workspace_size", n_cap, n_seg)
    ws = _ws(nb, dev, ws, stream)
    L = layout_struct(layout)
    _call("kpa_median_by_key", _p(keys), _p(rids), _p(seg_off), n_seg, n_cap, _p(rows), C.byref(L),
          _p(gkey), _p(gmed), _p(gseg), _p(o.get("cnt")), _p(o.get("sum")), _p(ws),
          ws.numel() * ws.element_size(), _stream(stream))
    return gkey, gmed, gseg


def kpa_join(lk, lr, l_seg_off, rk, rr, r_seg_off, rows_l, rows_r, layout, pairs_cap=0,
             nl_cap=None, nr_cap=None, ws=None, stream=None, outs=None):
    n_seg = l_seg_off.numel() - 1
    nl_cap = lk.numel() if nl_cap is None else nl_cap
    nr_cap = rk.numel() if nr_cap is None else nr_cap
    dev = lk.device
    o = outs or {}
    count = o["count"] if "count" in o else torch.empty(n_seg, dtype=torch.int64, device=dev)
    sumprod = o["sumprod"] if "sumprod" in o else torch.empty(n_seg, dtype=torch.int64,
                                                               device=dev)
    pairs = None
    if pairs_cap:
        pairs = o["pairs"] if "pairs" in o else torch.empty((max(pairs_cap, 1), 3),
                                                            dtype=torch.int64, device=dev)
    npairs = o["npairs"] if "npairs" in o else torch.empty(1, dtype=torch.int64, device=dev)
    nb = _ws_size("kpa_join_workspace_size", nl_cap, nr_cap, n_seg)
    ws = _ws(nb, dev, ws, stream)
    L = layout_struct(layout)
    _call("kpa_join", _p(lk), _p(lr), _p(l_seg_off), nl_cap, _p(rk), _p(rr), _p(r_seg_off), nr_cap,
          n_seg, _p(rows_l), _p(rows_r), C.byref(L), _p(count), _p(sumprod), _p(pairs), pairs_cap,
          _p(npairs), _p(ws), ws.numel() * ws.element_size(), _stream(stream))
    return count, sumprod, pairs, npairs


def kpa_join_runs(l_gkey, l_cnt, l_sum, l_gseg_off, r_gkey, r_cnt, r_sum, r_gseg_off,
                  gl_cap=None, gr_cap=None, ws=None, stream=None, outs=None):
    """Per-segment pair count and sum of value products from two run lists
    (key, count, sum per group); returns (count, sumprod)."""
    n_seg = l_gseg_off.numel() - 1
    gl_cap = l_gkey.numel() if gl_cap is None else gl_cap
    gr_cap = r_gkey.numel() if gr_cap is None else gr_cap
    dev = l_gkey.device
    o = outs or {}
    count = o["count"] if "count" in o else torch.empty(n_seg, dtype=torch.int64, device=dev)
    sumprod = o["sumprod"] if "sumprod" in o else torch.empty(n_seg, dtype=torch.int64,
                                                               device=dev)
    nb = _ws_size("kpa_join_runs_workspace_size", gl_cap, gr_cap, n_seg)
    ws = _ws(nb, dev, ws, stream)
    _call("kpa_join_runs", _p(l_gkey), _p(l_cnt), _p(l_sum), _p(l_gseg_off), gl_cap, _p(r_gkey),
          _p(r_cnt), _p(r_sum), _p(r_gseg_off), gr_cap, n_seg, _p(count), _p(sumprod), _p(ws),
          ws.numel() * ws.element_size(), _stream(stream))
    return count, sumprod


def kpa_materialize(rids, rows, row_bytes, out_rows=None, stream=None):
    n = rids.numel()
    dev = rids.device
    if out_rows is None:
        out_rows = torch.empty(max(n, 1) * row_bytes // 8, dtype=torch.int64, device=dev)
    _call("kpa_materialize", _p(rids), n, _p(rows), row_bytes, _p(out_rows), _stream(stream))
    return out_rows


def kpa_last_hip_error():
    return int(_lib.kpa_last_hip_error())


def kpa_materialize_extract(rids, rows, row_bytes, key_off, rid_base=0, out_rows=None,
                            out_keys=None, out_rids=None, stream=None):
    """Returns (out_rows, keys, rids): rows in KPA order and the KPA on the column at
    key_off of the emitted rows."""
    n = rids.numel()
    dev = rids.device
    if out_rows is None:
        out_rows = torch.empty(max(n, 1) * row_bytes // 8, dtype=torch.int64, device=dev)
    out_keys = torch.empty(max(n, 1), dtype=torch.int64, device=dev) if out_keys is None else out_keys
    out_rids = torch.empty(max(n, 1), dtype=torch.int32, device=dev) if out_rids is None else out_rids
    _call("kpa_materialize_extract", _p(rids), n, _p(rows), row_bytes, key_off, rid_base,
          _p(out_rows), _p(out_keys), _p(out_rids), _stream(stream))
    return out_rows, out_keys, out_rids


def kpa_keyswap(rids, rows, row_bytes, col_off, col_w=8, out_keys=None, stream=None):
    n = rids.numel()
    out_keys = torch.empty(max(n, 1), dtype=torch.int64, device=rids.device) \
        if out_keys is None else out_keys
    _call("kpa_keyswap", _p(rids), n, _p(rows), row_bytes, col_off, col_w, _p(out_keys),
          _stream(stream))
    return out_keys


def kpa_key_update(keys, table_keys, table_vals, n=None, out_missing=None, stream=None):
    """Updates keys in place from the sorted table; returns the device count of misses."""
    n = keys.numel() if n is None else n
    out_missing = torch.empty(1, dtype=torch.int64, device=keys.device) \
        if out_missing is None else out_missing
    _call("kpa_key_update", _p(keys), n, _p(table_keys), _p(table_vals), table_keys.numel(),
          _p(out_missing), _stream(stream))
    return out_missing


def kpa_key_writeback(keys, rids, rows, row_bytes, col_off, n=None, stream=None):
    n = keys.numel() if n is None else n
    _call("kpa_key_writeback", _p(keys), _p(rids), n, _p(rows), row_bytes, col_off,
          _stream(stream))


def kpa_select(keys, rids, seg_off, num_lo, num_hi=None, den=None, op=">", column=KPA_SEL_KEY,
               rows=None, layout=None, n_cap=None, outs=None, ws=None, stream=None):
    """Survivors of x * den[s] <op> num[s] per segment: (keys, rids, seg_off)."""
    n_seg = seg_off.numel() - 1
    n_cap = keys.numel() if n_cap is None else n_cap
    dev = keys.device
    o = outs or {}
    ok = o["keys"] if "keys" in o else torch.empty(max(n_cap, 1), dtype=torch.int64, device=dev)
    orr = o["rids"] if "rids" in o else torch.empty(max(n_cap, 1), dtype=torch.int32, device=dev)
    oo = o["seg_off"] if "seg_off" in o else torch.empty(n_seg + 1, dtype=torch.int64,
                                                         device=dev)
    ws = _ws(_ws_size("kpa_select_workspace_size", n_cap, n_seg), dev, ws, stream)
    L = layout_struct(layout) if layout is not None else None
    _call("kpa_select", _p(keys), _p(rids), _p(seg_off), n_seg, n_cap, _p(rows),
          C.byref(L) if L is not None else None, column, SELECT_OPS.get(op, op), _p(num_lo),
          _p(num_hi), _p(den), _p(ok), _p(orr), _p(oo), _p(ws), ws.numel() * ws.element_size(),
          _stream(stream))
    return ok, orr, oo


def kpa_reduce_all_windows(rows, layout, win_len, n_win, win_origin=0, n=None, outs=None,
                           ws=None, stream=None):
    """Per window: dict of cnt, sum_lo, sum_hi, max (device int64 [n_win]) and oob."""
    n = rows_count(rows, layout) if n is None else n
    dev = rows.device
    o = dict(outs or {})
    for name in ("cnt", "sum_lo", "sum_hi", "max"):
        if name not in o:
            o[name] = torch.empty(n_win, dtype=torch.int64, device=dev)
    if "oob" not in o:
        o["oob"] = torch.empty(1, dtype=torch.int64, device=dev)
    ws = _ws(_ws_size("kpa_reduce_all_windows_workspace_size", n_win), dev, ws, stream)
    L = layout_struct(layout)
    _call("kpa_reduce_all_windows", _p(rows), n, C.byref(L), win_len, win_origin, n_win,
          _p(o["cnt"]), _p(o["sum_lo"]), _p(o["sum_hi"]), _p(o["max"]), _p(o["oob"]), _p(ws),
          ws.numel() * ws.element_size(), _stream(stream))
    return o


def kpa_topk_per_key(keys, rids, seg_off, rows, layout, k, n_cap=None, outs=None, ws=None,
                     stream=None):
    """Returns dict gkey, gcnt, gstart, topv, gseg_off (device)."""
    n_seg = seg_off.numel() - 1
    n_cap = keys.numel() if n_cap is None else n_cap
    dev = keys.device
    cap = max(n_cap, 1)
    o = dict(outs or {})
    for name in ("gkey", "gcnt", "gstart", "topv"):
        if name not in o:
            o[name] = torch.empty(cap, dtype=torch.int64, device=dev)
    if "gseg_off" not in o:
        o["gseg_off"] = torch.empty(n_seg + 1, dtype=torch.int64, device=dev)
    ws = _ws(_ws_size("kpa_run_stats_workspace_size", n_cap, n_seg), dev, ws, stream)
    L = layout_struct(layout)
    _call("kpa_topk_per_key", _p(keys), _p(rids), _p(seg_off), n_seg, n_cap, _p(rows), C.byref(L),
          k, _p(o["gkey"]), _p(o["gcnt"]), _p(o["gstart"]), _p(o["topv"]), _p(o["gseg_off"]),
          _p(ws), ws.numel() * ws.element_size(), _stream(stream))
    return o


def kpa_unique_count_by_key(keys, rids, seg_off, rows, layout, n_cap=None, outs=None, ws=None,
                            stream=None):
    """Returns dict gkey, uniq, gseg_off (device)."""
    n_seg = seg_off.numel() - 1
    n_cap = keys.numel() if n_cap is None else n_cap
    dev = keys.device
    cap = max(n_cap, 1)
    o = dict(outs or {})
    for name in ("gkey", "uniq"):
        if name not in o:
            o[name] = torch.empty(cap, dtype=torch.int64, device=dev)
    if "gseg_off" not in o:
        o["gseg_off"] = torch.empty(n_seg + 1, dtype=torch.int64, device=dev)
    ws = _ws(_ws_size("kpa_run_stats_workspace_size", n_cap, n_seg), dev, ws, stream)
    L = layout_struct(layout)
    _call("kpa_unique_count_by_key", _p(keys), _p(rids), _p(seg_off), n_seg, n_cap, _p(rows),
          C.byref(L), _p(o["gkey"]), _p(o["uniq"]), _p(o["gseg_off"]), _p(ws),
          ws.numel() * ws.element_size(), _stream(stream))
    return o


def kpa_sort_rows_windowed(rows, layout, win_len, n_win, win_origin=0, n=None, out_rows=None,
                           out_win_off=None, out_oob=None, ws=None, stream=None):
    """Rows ordered by (window, key) stably, moving whole rows: (out_rows, win_off, oob)."""
    n = rows_count(rows, layout) if n is None else n
    dev = rows.device
    if out_rows is None:
        out_rows = torch.empty(max(n, 1) * layout.row_bytes // 8, dtype=torch.int64, device=dev)
    out_win_off = (torch.empty(n_win + 1, dtype=torch.int64, device=dev)
                   if out_win_off is None else out_win_off)
    out_oob = torch.empty(1, dtype=torch.int64, device=dev) if out_oob is None else out_oob
    nb = C.c_size_t(0)
    _call("kpa_sort_rows_windowed_workspace_size", n, layout.row_bytes, C.byref(nb))
    ws = _ws(int(nb.value), dev, ws, stream)
    L = layout_struct(layout)
    _call("kpa_sort_rows_windowed", _p(rows), n, C.byref(L), win_len, win_origin, n_win,
          _p(out_rows), _p(out_win_off), _p(out_oob), _p(ws), ws.numel() * ws.element_size(),
          _stream(stream))
    return out_rows, out_win_off, out_oob


def kpa_hash_groupby(rows, layout, table_cap, g_cap=None, n=None, outs=None, ws=None,
                     stream=None):
    """Groups in table order: dict gkey, cnt, sum, max (device, g_cap) and ngroups."""
    n = rows_count(rows, layout) if n is None else n
    dev = rows.device
    g_cap = table_cap + 1 if g_cap is None else g_cap
    o = dict(outs or {})
    for name in ("gkey", "cnt", "sum", "max"):
        if name not in o:
            o[name] = torch.empty(max(g_cap, 1), dtype=torch.int64, device=dev)
    if "ngroups" not in o:
        o["ngroups"] = torch.empty(1, dtype=torch.int64, device=dev)
    ws = _ws(_ws_size("kpa_hash_groupby_workspace_size", table_cap), dev, ws, stream)
    L = layout_struct(layout)
    _call("kpa_hash_groupby", _p(rows), n, C.byref(L), table_cap, _p(o["gkey"]), _p(o["cnt"]),
          _p(o["sum"]), _p(o["max"]), g_cap, _p(o["ngroups"]), _p(ws),
          ws.numel() * ws.element_size(), _stream(stream))
    return o


def kpa_window_panes(gkey, gseg_off, panes_per_window, out_cap, outs=None, stream=None):
    """(keys, rids, seg_off) of the sliding windows' concatenated pane groups."""
    n_pane = gseg_off.numel() - 1
    n_win = n_pane - panes_per_window + 1
    dev = gkey.device
    o = outs or {}
    ok = o["keys"] if "keys" in o else torch.empty(max(out_cap, 1), dtype=torch.int64, device=dev)
    orr = o["rids"] if "rids" in o else torch.empty(max(out_cap, 1), dtype=torch.int32,
                                                    device=dev)
    oo = o["seg_off"] if "seg_off" in o else torch.empty(n_win + 1, dtype=torch.int64,
                                                         device=dev)
    _call("kpa_window_panes", _p(gkey), _p(gseg_off), n_pane, panes_per_window, _p(ok), _p(orr),
          _p(oo), out_cap, _stream(stream))
    return ok, orr, oo


def kpa_partition_kpa(keys, rids, win_len, n_win, win_origin=0, n=None, out_keys=None,
                      out_rids=None, out_win_off=None, out_oob=None, ws=None, stream=None):
    n = keys.numel() if n is None else n
    dev = keys.device
    out_keys = torch.empty(max(n, 1), dtype=torch.int64, device=dev) if out_keys is None else out_keys
    out_rids = torch.empty(max(n, 1), dtype=torch.int32, device=dev) if out_rids is None else out_rids
    out_win_off = (torch.empty(n_win + 1, dtype=torch.int64, device=dev)
                   if out_win_off is None else out_win_off)
    out_oob = torch.empty(1, dtype=torch.int64, device=dev) if out_oob is None else out_oob
    ws = _ws(_ws_size("kpa_partition_windows_workspace_size", n, n_win), dev, ws, stream)
    _call("kpa_partition_kpa", _p(keys), _p(rids), n, win_len, win_origin, n_win, _p(out_keys),
          _p(out_rids), _p(out_win_off), _p(out_oob), _p(ws), ws.numel() * ws.element_size(),
          _stream(stream))
    return out_keys, out_rids, out_win_off, out_oob


def new_models(n, device):
    """Uninitialised kpa_pwl_model array (bytes) for n segments."""
    return torch.zeros(n * PWL_MODEL_BYTES, dtype=torch.uint8, device=device)


def kpa_pwl_fit(sorted_keys, seg_off, n_seg_model=1024, models=None, stream=None):
    n_seg = seg_off.numel() - 1
    models = new_models(n_seg, sorted_keys.device) if models is None else models
    _call("kpa_pwl_fit", _p(sorted_keys), _p(seg_off), n_seg, n_seg_model, _p(models),
          _stream(stream))
    return models


def model_fields(models):
    """Host view of a models buffer: list of (kmin, kmax, n_seg, knots)."""
    raw = models.detach().cpu().numpy().tobytes()
    import numpy as np
    out = []
    for i in range(len(raw) // PWL_MODEL_BYTES):
        b = raw[i * PWL_MODEL_BYTES:(i + 1) * PWL_MODEL_BYTES]
        kmin = int.from_bytes(b[0:8], "little")
        kmax = int.from_bytes(b[8:16], "little")
        ns = int.from_bytes(b[16:20], "little")
        knots = np.frombuffer(b[24:24 + 4 * (KPA_PWL_MAX_SEG + 1)], dtype=np.float32)
        out.append((kmin, kmax, ns, knots[:ns + 1].copy()))
    return out


def new_sort_stats(device):
    return torch.zeros(SORT_STATS_WORDS, dtype=torch.int64, device=device)


def kpa_mlp_training_set(sorted_keys, S, model, stream=None):
    dev = sorted_keys.device
    x = torch.empty(S, dtype=torch.float32, device=dev)
    y = torch.empty(S, dtype=torch.float32, device=dev)
    _call("kpa_mlp_training_set", _p(sorted_keys), sorted_keys.numel(), S, _p(x), _p(y), _p(model),
          _stream(stream))
    return x, y


def kpa_mlp_forward(params, x, stream=None):
    out = torch.empty_like(x)
    _call("kpa_mlp_forward", _p(params), _p(x), x.numel(), _p(out), _stream(stream))
    return out


def kpa_mlp_loss_grad(params, x, y, ws=None, stream=None):
    m = x.numel()
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    grad = torch.empty(KPA_MLP_PARAMS, dtype=torch.float32, device=x.device)
    nb = _ws_size("kpa_mlp_loss_grad_workspace_size", m)
    ws = _ws(nb, x.device, ws, stream)
    _call("kpa_mlp_loss_grad", _p(params), _p(x), _p(y), m, _p(loss), _p(grad), _p(ws),
          ws.numel() * ws.element_size(), _stream(stream))
    return loss, grad


def kpa_mlp_adam_step(params, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                      stream=None):
    _call("kpa_mlp_adam_step", _p(params), _p(grad), _p(m), _p(v), t, lr, beta1, beta2, eps,
          _stream(stream))


def kpa_mlp_train(params, m, v, x, y, t0, steps, lr=1e-3, ws=None, stream=None):
    n = x.numel()
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    nb = _ws_size("kpa_mlp_loss_grad_workspace_size", n) + 4 * KPA_MLP_PARAMS + 512
    ws = _ws(nb, x.device, ws, stream)
    _call("kpa_mlp_train", _p(params), _p(m), _p(v), _p(x), _p(y), n, t0, steps, lr, _p(loss),
          _p(ws), ws.numel() * ws.element_size(), _stream(stream))
    return loss


def kpa_mlp_init(uniforms, params=None, stream=None):
    """Starting parameters of the network from KPA_MLP_PARAMS uniforms."""
    if uniforms.dtype != torch.float32 or uniforms.numel() < KPA_MLP_PARAMS:
        raise ValueError(f"need {KPA_MLP_PARAMS} float32 uniforms")
    params = torch.empty(KPA_MLP_PARAMS, dtype=torch.float32, device=uniforms.device) \
        if params is None else params
    _call("kpa_mlp_init", _p(uniforms), _p(params), _stream(stream))
    return params


def kpa_mlp_to_pwl(params, model, n_seg_model=1024, stream=None):
    _call("kpa_mlp_to_pwl", _p(params), n_seg_model, _p(model), _stream(stream))
    return model


# ---------------------------------------------------------------- serving --

def kpa_ingest_bundle(host_rows, layout, dev_rows, ts_add=0, stream=None):
    n = rows_count(host_rows, layout)
    L = layout_struct(layout)
    _call("kpa_ingest_bundle", C.c_void_p(host_rows.data_ptr()), n, C.byref(L), ts_add,
          _p(dev_rows), _stream(stream))


def kpa_balance_knob_update(k_low, k_high, hbm_util, bw_util, delay_ms, target_ms):
    """The knob after one refresh: (k_low, k_high)."""
    lo, hi = C.c_double(k_low), C.c_double(k_high)
    _call("kpa_balance_knob_update", C.byref(lo), C.byref(hi), hbm_util, bw_util, delay_ms,
          target_ms)
    return lo.value, hi.value


def _ts_column(rows, layout):
    import numpy as np
    a = rows.numpy() if hasattr(rows, "numpy") else rows
    b = a.view(np.uint8).reshape(-1, layout.row_bytes)
    w = layout.ts_w
    col = b[:, layout.ts_off:layout.ts_off + w].copy().view(np.uint64 if w == 8 else np.uint32)
    return col.reshape(-1)


class Server:
    """The serving loop (kpa_server_*).  Bundles are host tensors (pinned for
    asynchronous copies) that the server reads until drain(); this object
    keeps them alive until then."""

    def __init__(self, **cfg):
        c = kpa_server_config()
        _call("kpa_server_config_default", C.byref(c))
        for k, v in cfg.items():
            setattr(c, k, float(v) if k in ("target_delay_ms", "host_bw_gbs") else int(v))
        self.cfg = c
        h = C.c_void_p(None)
        _call("kpa_server_create", C.byref(c), C.byref(h))
        self.h = h
        self._keep = []
        self._layouts = {}

    def add_query(self, kind, layout, win_len, win_origin=0):
        q = C.c_uint32(0)
        L = layout_struct(layout)
        _call("kpa_server_add_query", self.h, kind, C.byref(L), win_len, win_origin, C.byref(q))
        self._layouts[q.value] = layout
        return q.value

    def submit(self, qid, rows, side=0, ts_base=0, ts_lo=None, ts_hi=None, blocking=True):
        lay = self._layouts[qid]
        n = rows_count(rows, lay)
        if n == 0:
            return
        if ts_lo is None or ts_hi is None:
            ts = _ts_column(rows, lay)
            ts_lo, ts_hi = int(ts.min()), int(ts.max())
        self._keep.append(rows)
        _call("kpa_server_submit", self.h, qid, side, C.c_void_p(rows.data_ptr()), n, ts_base,
              ts_lo, ts_hi, 1 if blocking else 0)

    def watermark(self, qid, t):
        _call("kpa_server_watermark", self.h, qid, t)

    def poll(self, timeout_ms=0):
        """One finished window result (dict) or None; with keep_groups the
        per-key arrays come as numpy uint64 arrays under "arrays" (SUM: gkey,
        cnt, sum, max; MEDIAN: gkey, median) and the server's copy is freed."""
        r = kpa_window_result()
        got = C.c_int32(0)
        _call("kpa_server_poll", self.h, C.byref(r), C.byref(got), timeout_ms)
        if not got.value:
            return None
        d = r.as_dict()
        if r.groups_data and r.groups_words:
            import numpy as np
            flat = np.ctypeslib.as_array(r.groups_data, shape=(r.groups_words,)).copy()
            names = ("gkey", "cnt", "sum", "max") if r.kind == KPA_Q_SUM else ("gkey", "median")
            G = r.groups
            d["arrays"] = {nm: flat[i * G:(i + 1) * G] for i, nm in enumerate(names)}
            _call("kpa_server_release_groups", self.h, r.groups_data)
        return d

    def trace(self, cap=65536):
        buf = (kpa_monitor_sample * cap)()
        n = C.c_uint32(0)
        _call("kpa_server_trace", self.h, buf, cap, C.byref(n))
        return [buf[i].as_dict() for i in range(n.value)]

    def results(self):
        out = []
        while True:
            r = self.poll(0)
            if r is None:
                return out
            out.append(r)

    def drain(self, timeout_ms=-1):
        _call("kpa_server_drain", self.h, timeout_ms)
        self._keep.clear()

    def stats(self):
        st = kpa_server_statistics()
        _call("kpa_server_stats", self.h, C.byref(st))
        return st.as_dict()

    def close(self):
        if self.h:
            _call("kpa_server_destroy", self.h)
            self.h = C.c_void_p(None)
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
        return False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
