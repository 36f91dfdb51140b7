"""The C-ABI library loads and exports every function include/kpa.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kpa.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:kpa_status|int32_t|const char\*)\s+(kpa_\w+)\s*\(", src, re.M)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = declared()
    assert "kpa_sort_segmented" in names and "kpa_partition_windows" in names
    assert len(names) >= 25


def test_library_exports_every_declared_symbol():
    import paper_1901_01328_amd as P
    assert os.path.exists(P.LIB_PATH), "libkpa.so not built"
    lib = ctypes.CDLL(P.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


def test_binding_covers_every_symbol():
    import paper_1901_01328_amd as P
    k = P.load()
    missing = [n for n in declared() if n not in k.EXPORTED]
    assert not missing, f"binding lacks: {missing}"


def test_host_side_errors_without_gpu():
    """Argument checks run on the host and return codes without touching a GPU."""
    import paper_1901_01328_amd as P
    k = P.load()
    lib = k._lib
    n = ctypes.c_size_t(0)
    assert lib.kpa_sort_workspace_size(1 << 20, 1, 0, ctypes.byref(n)) == 0 and n.value > 0
    assert lib.kpa_sort_workspace_size(1 << 20, 1, 7, ctypes.byref(n)) == k.KPA_EINVAL
    L = k.kpa_row_layout(32, 0, 8, 8, 16, 8)
    # n_win out of range, before anything is enqueued
    rc = lib.kpa_partition_windows(None, 0, ctypes.byref(L), 10, 0, 0, 0, None, None, None, None,
                                   None, None, 0, None)
    assert rc == k.KPA_EUNSUPPORTED
    bad = k.kpa_row_layout(30, 0, 8, 8, 16, 8)
    rc = lib.kpa_extract(None, 5, ctypes.byref(bad), 0, None, None, None, None)
    assert rc == k.KPA_EINVAL
    assert b"row_bytes" in lib.kpa_last_error_string()
    rc = lib.kpa_topk_by_sum(None, None, None, 1, 10, 17, None, None, None, None, 0, None)
    assert rc == k.KPA_EUNSUPPORTED
    # batch configuration: the learned path's mean bucket size 2^bucket_log2
    cfg = k.kpa_batch_config()
    assert lib.kpa_batch_config_default(k.KPA_SORT_LEARNED, ctypes.byref(cfg)) == 0
    assert cfg.bucket_log2 == 0
    for bl, want in ((0, 0), (6, 0), (12, 0), (5, k.KPA_EINVAL), (13, k.KPA_EINVAL)):
        cfg.bucket_log2 = bl
        assert lib.kpa_batch_sort_workspace_size(1 << 20, 4, ctypes.byref(cfg),
                                                 ctypes.byref(n)) == want, bl
    assert b"bucket_log2" in lib.kpa_last_error_string()
    # run-list join: pointers and sizes are checked before anything is enqueued
    fake = ctypes.c_void_p(1 << 20)          # aligned, never dereferenced on these paths
    rc = lib.kpa_join_runs(fake, fake, fake, fake, 10, fake, fake, fake, fake, 10, 2, None, fake,
                           fake, 1 << 20, None)
    assert rc == k.KPA_EINVAL
    rc = lib.kpa_join_runs(fake, fake, fake, fake, 1 << 32, fake, fake, fake, fake, 10, 2, fake,
                           fake, fake, 1 << 20, None)
    assert rc == k.KPA_EUNSUPPORTED
    rc = lib.kpa_join_runs(fake, fake, fake, fake, 1000, fake, fake, fake, fake, 1000, 2, fake,
                           fake, fake, 16, None)
    assert rc == k.KPA_EWORKSPACE
    assert lib.kpa_join_runs_workspace_size(1000, 1000, 2, ctypes.byref(n)) == 0 and n.value > 16


def test_server_config_checked_on_the_host():
    """Invalid serving configurations are refused before any device call."""
    import paper_1901_01328_amd as P
    k = P.load()
    lib = k._lib
    cfg = k.kpa_server_config()
    assert lib.kpa_server_config_default(ctypes.byref(cfg)) == 0
    assert cfg.budget_bytes == 64 << 30 and cfg.slots == 8
    h = ctypes.c_void_p(None)
    bad = k.kpa_server_config.from_buffer_copy(cfg)
    bad.slots = 0
    assert lib.kpa_server_create(ctypes.byref(bad), ctypes.byref(h)) == k.KPA_EINVAL
    bad = k.kpa_server_config.from_buffer_copy(cfg)
    bad.budget_bytes = 1 << 20          # cannot hold the slots' scratch
    assert lib.kpa_server_create(ctypes.byref(bad), ctypes.byref(h)) == k.KPA_EBUDGET
    assert b"budget" in lib.kpa_last_error_string()
    assert not h.value
