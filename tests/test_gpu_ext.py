"""GPU parity of the single-pass benchmarks and the remaining Table 2
primitives against the CPU oracle, element by element, through the C ABI:
top-k values per key, unique count per key, the unkeyed window reduction
(exact 128-bit sums), Select with exact ratio thresholds, the windowed filter,
KeySwap, key update and write-back, Materialize with Extract, partition of a
KPA, sliding windows from panes, and inputs beyond 2^30 entries."""
import numpy as np
import pytest
import torch

import datagen
from datagen.rows import LAYOUT16, LAYOUT32, RowLayout
from gpu_util import dev_u32, dev_u64, kpa_mod, need_gpu, say, u32, u64

pytestmark = pytest.mark.gpu
M64 = (1 << 64) - 1


@pytest.fixture(scope="module")
def K():
    need_gpu()
    return kpa_mod()


def rows32(key, val, ts, pad=None):
    n = len(key)
    a = np.zeros((n, 4), np.uint64)
    a[:, 0], a[:, 1], a[:, 2] = key, val, ts
    a[:, 3] = np.arange(n, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15) if pad is None else pad
    return a


def dev_rows(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).to("cuda")


def run_sizes_keys(rng, n, n_seg):
    """Keys whose runs span every size class: many short runs, some of a few
    hundred to 4096 entries, and a few longer than 4096 (big class)."""
    pool = rng.integers(0, 1 << 63, size=4000, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    w = np.concatenate([np.full(3, 2000.0), np.full(30, 60.0), np.full(3967, 1.0)])
    k = rng.choice(pool, size=n, p=w / w.sum())
    k[:5] = np.uint64(0)
    k[5:9] = np.uint64(M64)
    cuts = np.sort(rng.integers(0, n + 1, size=n_seg - 1))
    off = np.concatenate([[0], cuts, [n]]).astype(np.uint64)
    return k, off


def sorted_kpa(K, orc, keys, off):
    rids = np.arange(len(keys), dtype=np.uint32)
    sk, sr = orc.sort_segmented(keys, rids, off)
    return sk, sr


# ------------------------------------------------------ per-key statistics --

@pytest.mark.parametrize("case", ["u64_wide", "u64_repeats", "u32_values"])
def test_topk_and_unique_per_key(K, orc, case):
    rng = np.random.default_rng({"u64_wide": 1, "u64_repeats": 2, "u32_values": 3}[case])
    n, n_seg = 150_000, 5
    keys, off = run_sizes_keys(rng, n, n_seg)
    off[2] = off[1]                                      # an empty segment
    if case == "u32_values":
        lay = LAYOUT16
        vals = rng.integers(0, 1 << 32, size=n, dtype=np.uint64)
        vals[rng.random(n) < 0.1] = np.uint64(0xFFFFFFFF)
        raw = np.zeros((n, 2), np.uint64)
        raw[:, 0] = keys
        raw[:, 1] = vals  # value u32 at 8, timestamp u32 at 12 (0)
    else:
        lay = LAYOUT32
        hi = 1 << 64 if case == "u64_wide" else 7
        vals = rng.integers(0, min(hi, 1 << 63), size=n, dtype=np.uint64)
        if case == "u64_wide":
            vals |= rng.integers(0, 2, size=n, dtype=np.uint64) << np.uint64(63)
            vals[rng.random(n) < 0.05] = np.uint64(M64)
        raw = rows32(keys, vals, np.zeros(n, np.uint64))
    sk, sr = sorted_kpa(K, orc, keys, off)
    d_rows = dev_rows(raw)
    dk, dr, doff = dev_u64(sk), dev_u32(sr), dev_u64(off)
    for k in (1, 5, 16):
        say(f"topk_per_key {case} k={k}")
        o = K.kpa_topk_per_key(dk, dr, doff, d_rows, lay, k)
        torch.cuda.synchronize()
        gs = u64(o["gseg_off"])
        gkey, gcnt, gstart, topv = u64(o["gkey"]), u64(o["gcnt"]), u64(o["gstart"]), u64(o["topv"])
        for s in range(n_seg):
            a, b = int(off[s]), int(off[s + 1])
            ek, ec, etn, etv = orc.topk_per_key(sk[a:b], sr[a:b], raw, lay, k)
            g0, g1 = int(gs[s]), int(gs[s + 1])
            assert g1 - g0 == len(ek)
            assert np.array_equal(gkey[g0:g1], ek) and np.array_equal(gcnt[g0:g1], ec)
            assert np.array_equal(gstart[g0:g1] - np.uint64(a),
                                  np.cumsum(np.concatenate([[0], ec]))[:-1].astype(np.uint64))
            for i in range(len(ek)):
                t = int(etn[i])
                st = int(gstart[g0 + i])
                assert np.array_equal(topv[st:st + t], etv[i, :t]), (s, i, k)
        if k == 16:
            assert int(gcnt[:int(gs[-1])].max()) > 4096  # the big class took part
    say(f"unique_count {case}")
    o = K.kpa_unique_count_by_key(dk, dr, doff, d_rows, lay)
    torch.cuda.synchronize()
    gs = u64(o["gseg_off"])
    for s in range(n_seg):
        a, b = int(off[s]), int(off[s + 1])
        ek, eu = orc.unique_count_by_key(sk[a:b], sr[a:b], raw, lay)
        g0, g1 = int(gs[s]), int(gs[s + 1])
        assert np.array_equal(u64(o["gkey"])[g0:g1], ek)
        assert np.array_equal(u64(o["uniq"])[g0:g1], eu)


def test_run_stats_empty_and_k_range(K):
    z = torch.zeros(1, dtype=torch.int64, device="cuda")
    off = dev_u64([0, 0, 0])
    o = K.kpa_topk_per_key(z, torch.zeros(1, dtype=torch.int32, device="cuda"), off,
                           torch.zeros(4, dtype=torch.int64, device="cuda"), LAYOUT32, 3, n_cap=0)
    torch.cuda.synchronize()
    assert u64(o["gseg_off"]).tolist() == [0, 0, 0]
    with pytest.raises(K.KpaError):
        K.kpa_topk_per_key(z, torch.zeros(1, dtype=torch.int32, device="cuda"), off, z, LAYOUT32,
                           17, n_cap=0)


# -------------------------------------------------------- unkeyed reduce ---

@pytest.mark.parametrize("seed", [0, 1])
def test_reduce_all_windows(K, orc, seed):
    rng = np.random.default_rng(20 + seed)
    n, W, nw, origin = 300_001, 1000, 37, 5000
    ts = rng.integers(0, origin + W * nw + 3000, size=n, dtype=np.uint64)
    vals = rng.integers(0, 1 << 63, size=n, dtype=np.uint64) | (
        rng.integers(0, 2, size=n, dtype=np.uint64) << np.uint64(63))
    vals[rng.random(n) < 0.3] = np.uint64(M64)          # sums far past 2^64
    keys = rng.integers(0, 50, size=n, dtype=np.uint64)
    raw = rows32(keys, vals, ts)
    o = K.kpa_reduce_all_windows(dev_rows(raw), LAYOUT32, W, nw, win_origin=origin)
    torch.cuda.synchronize()
    c, lo, hi, mx, oob = orc.reduce_all_windows(raw, LAYOUT32, W, nw, origin)
    assert np.array_equal(u64(o["cnt"]), c) and np.array_equal(u64(o["sum_lo"]), lo)
    assert np.array_equal(u64(o["sum_hi"]), hi) and np.array_equal(u64(o["max"]), mx)
    assert int(o["oob"].item()) == oob and int(hi.max()) > 0


def test_reduce_all_u32_columns(K, orc):
    rng = np.random.default_rng(25)
    n = 70_000
    raw = np.zeros((n, 2), np.uint64)
    raw[:, 0] = rng.integers(0, 9, size=n, dtype=np.uint64)
    v = rng.integers(0, 1 << 32, size=n, dtype=np.uint64)
    t = np.sort(rng.integers(0, 1000, size=n, dtype=np.uint64))
    raw[:, 1] = v | (t << np.uint64(32))
    o = K.kpa_reduce_all_windows(dev_rows(raw), LAYOUT16, 100, 10)
    torch.cuda.synchronize()
    c, lo, hi, mx, oob = orc.reduce_all_windows(raw, LAYOUT16, 100, 10)
    assert np.array_equal(u64(o["cnt"]), c) and np.array_equal(u64(o["sum_lo"]), lo)
    assert np.array_equal(u64(o["sum_hi"]), hi) and np.array_equal(u64(o["max"]), mx)


# ------------------------------------------------------------------ select --

@pytest.mark.parametrize("op", [">", ">=", "<", "<=", "==", "!="])
@pytest.mark.parametrize("column", [0, 1])
def test_select(K, orc, op, column):
    rng = np.random.default_rng(30 + column * 7 + len(op))
    n, n_seg = 90_001, 7
    keys = rng.integers(0, 200, size=n, dtype=np.uint64) * np.uint64(0x0123456789AB)
    vals = rng.integers(0, 1 << 63, size=n, dtype=np.uint64)
    raw = rows32(keys, vals, np.zeros(n, np.uint64))
    cuts = np.sort(rng.integers(0, n + 1, size=n_seg - 1))
    off = np.concatenate([[0], cuts, [n]]).astype(np.uint64)
    off[3] = off[2]
    rids = rng.permutation(n).astype(np.uint32)
    kk = keys[rids]
    num_lo, num_hi, den = [], [], []
    for s in range(n_seg):
        d = [1, 3, 0, 1 << 40, 7, 2, 1][s]
        a, b = int(off[s]), int(off[s + 1])
        if b > a:
            i = int(rng.integers(a, b))
            x = int(kk[i]) if column == 0 else int(vals[rids[i]])
            v = x * d
        else:
            v = 12345
        num_lo.append(v & M64)
        num_hi.append(v >> 64)
        den.append(d)
    say(f"select op={op} column={column}")
    ok, orr, oo = K.kpa_select(dev_u64(kk), dev_u32(rids), dev_u64(off), dev_u64(num_lo),
                               dev_u64(num_hi), dev_u64(den), op=op, column=column,
                               rows=dev_rows(raw), layout=LAYOUT32)
    torch.cuda.synchronize()
    ek, er, eo = orc.select(kk, rids, off, num_lo, num_hi, den, op, column, raw, LAYOUT32)
    assert np.array_equal(u64(oo), eo)
    m = int(eo[-1])
    assert np.array_equal(u64(ok)[:m], ek) and np.array_equal(u32(orr)[:m], er)


def test_windowed_filter(K, orc):
    """Sec. 6 Windowed Filter: A's exact window average filters B's keys
    (unkeyed reduce on A, partition of B, Select with the ratio threshold)."""
    rng = np.random.default_rng(40)
    na, nb, W, nw = 200_000, 170_000, 10 ** 6, 12
    va = rng.integers(0, 1 << 64, size=na, dtype=np.uint64)
    ra = rows32(rng.integers(0, 99, size=na, dtype=np.uint64), va,
                np.sort(rng.integers(0, W * nw, size=na, dtype=np.uint64)))
    kb = rng.integers(0, 1 << 64, size=nb, dtype=np.uint64)
    tb = np.sort(rng.integers(0, W * (nw + 1), size=nb, dtype=np.uint64))
    rb = rows32(kb, np.zeros(nb, np.uint64), tb)
    da, db = dev_rows(ra), dev_rows(rb)
    st = K.kpa_reduce_all_windows(da, LAYOUT32, W, nw)
    bk, br, boff, boob = K.kpa_partition_windows(db, LAYOUT32, W, nw)
    ok, orr, oo = K.kpa_select(bk, br, boff, st["sum_lo"], st["sum_hi"], st["cnt"], op=">",
                               column=K.KPA_SEL_KEY, n_cap=nb)
    torch.cuda.synchronize()
    ek, er, eo = orc.window_filter(ra, rb, LAYOUT32, W, nw)
    assert np.array_equal(u64(oo), eo)
    m = int(eo[-1])
    assert 0 < m < nb
    assert np.array_equal(u64(ok)[:m], ek) and np.array_equal(u32(orr)[:m], er)


# ------------------------------------------------ KeySwap, update, write-back --

def test_keyswap(K, orc):
    rng = np.random.default_rng(50)
    n = 40_000
    raw = rows32(rng.integers(0, 1 << 64, size=n, dtype=np.uint64),
                 rng.integers(0, 1 << 64, size=n, dtype=np.uint64),
                 rng.integers(0, 1 << 64, size=n, dtype=np.uint64))
    rids = rng.integers(0, n, size=77_777).astype(np.uint32)
    d = dev_rows(raw)
    for col_off, w in ((16, 8), (8, 8), (20, 4), (0, 4)):
        got = K.kpa_keyswap(dev_u32(rids), d, 32, col_off, w)
        torch.cuda.synchronize()
        assert np.array_equal(u64(got), orc.keyswap(rids, raw, 32, col_off, w)), (col_off, w)


@pytest.mark.parametrize("tn", [0, 1, 1000, 2048, 2049, 100_000])
def test_key_update(K, orc, tn):
    rng = np.random.default_rng(60 + tn)
    u = np.unique(rng.integers(0, 1 << 40, size=2 * tn + 1, dtype=np.uint64))
    tk = np.sort(u[rng.permutation(len(u))[:tn]])
    tv = rng.integers(0, 1 << 64, size=tn, dtype=np.uint64)
    n = 123_457
    keys = rng.integers(0, 1 << 40, size=n, dtype=np.uint64)
    if tn:
        hit = rng.random(n) < 0.8
        keys[hit] = tk[rng.integers(0, tn, size=int(hit.sum()))]
    keys[:3] = np.uint64(M64)
    dk = dev_u64(keys)
    miss = K.kpa_key_update(dk, dev_u64(tk), dev_u64(tv))
    torch.cuda.synchronize()
    ek, emiss = orc.key_update(keys, tk, tv)
    assert np.array_equal(u64(dk), ek) and int(miss.item()) == emiss


def test_key_writeback_then_keyswap(K, orc):
    rng = np.random.default_rng(70)
    n = 50_000
    raw = rows32(rng.integers(0, 1 << 64, size=n, dtype=np.uint64),
                 rng.integers(0, 1 << 64, size=n, dtype=np.uint64),
                 rng.integers(0, 1 << 64, size=n, dtype=np.uint64))
    rids = rng.permutation(n)[:30_000].astype(np.uint32)
    keys = rng.integers(0, 1 << 64, size=len(rids), dtype=np.uint64)
    d = dev_rows(raw)
    K.kpa_key_writeback(dev_u64(keys), dev_u32(rids), d, 32, 24)
    back = K.kpa_keyswap(dev_u32(rids), d, 32, 24, 8)
    torch.cuda.synchronize()
    exp = orc.key_writeback(keys, rids, raw, 32, 24)
    assert np.array_equal(d.cpu().numpy().view(np.uint8).reshape(-1), exp)
    assert np.array_equal(u64(back), keys)


@pytest.mark.parametrize("row_bytes,key_off", [(32, 16), (32, 8), (32, 0), (16, 8), (24, 16)])
def test_materialize_extract(K, orc, row_bytes, key_off):
    rng = np.random.default_rng(80 + row_bytes + key_off)
    n = 20_000
    raw = rng.integers(0, 1 << 64, size=n * row_bytes // 8, dtype=np.uint64)
    rids = rng.integers(0, n, size=33_333).astype(np.uint32)
    out, ok, orr = K.kpa_materialize_extract(dev_u32(rids), dev_u64(raw), row_bytes, key_off,
                                             rid_base=11)
    torch.cuda.synchronize()
    er, ek, err_ = orc.materialize_extract(rids, raw, row_bytes, key_off, rid_base=11)
    assert np.array_equal(out.cpu().numpy().view(np.uint8)[:len(rids) * row_bytes], er)
    assert np.array_equal(u64(ok)[:len(rids)], ek) and np.array_equal(u32(orr)[:len(rids)], err_)


# ------------------------------------------------------ partition of a KPA --

def test_partition_kpa(K, orc):
    rng = np.random.default_rng(90)
    n, W, nw, origin = 333_333, 777, 50, 1000
    ts = rng.integers(0, origin + W * nw + 500, size=n, dtype=np.uint64)
    rids = rng.permutation(n).astype(np.uint32)
    ok, orr, off, oob = K.kpa_partition_kpa(dev_u64(ts), dev_u32(rids), W, nw, win_origin=origin)
    torch.cuda.synchronize()
    # the oracle partitions 8-byte rows (the timestamps) and returns row indices
    lay8 = RowLayout(8, 0, 0, 8, 0, 8)
    ek, eidx, eoff, eoob = orc.partition(ts.view(np.uint8), lay8, W, nw, origin)
    assert np.array_equal(u64(off), eoff) and int(oob.item()) == eoob
    m = int(eoff[-1])
    assert np.array_equal(u64(ok)[:m], ek) and np.array_equal(u32(orr)[:m], rids[eidx])


# ------------------------------------------------------------ sliding windows --

def test_sliding_windows_from_panes(K, orc):
    """Sliding windows (length 3 slides) as panes: partition by the slide,
    sort and reduce each pane, concatenate the panes of each window, sort,
    and reduce the pane groups' count/sum/max columns."""
    from paper_1901_01328_amd.pipeline import SlidingAggregation
    rng = np.random.default_rng(100)
    n, S, P, n_win = 400_000, 10 ** 5, 3, 20
    keys = rng.integers(0, 3000, size=n, dtype=np.uint64) * np.uint64(0xABCDEF12345)
    vals = rng.integers(0, 1 << 64, size=n, dtype=np.uint64)
    ts = rng.integers(0, S * (n_win + P - 1) + 5 * S, size=n, dtype=np.uint64)
    raw = rows32(keys, vals, ts)
    agg = SlidingAggregation(n, LAYOUT32, S * P, S, n_win, device="cuda")
    agg.step(dev_rows(raw))
    torch.cuda.synchronize()
    ek, ec, es, em, eo = orc.sliding_aggregate(raw, LAYOUT32, S * P, S, n_win)
    go = u64(agg.wseg)
    assert np.array_equal(go, eo)
    g = int(eo[-1])
    assert np.array_equal(u64(agg.wkey)[:g], ek)
    assert np.array_equal(u64(agg.w["cnt"])[:g], ec)
    assert np.array_equal(u64(agg.w["sum"])[:g], es)
    assert np.array_equal(u64(agg.w["max"])[:g], em)


# ------------------------------------------------------- beyond 2^30 entries --

def test_partition_beyond_2_30_rows(K):
    """2^30 + 4097 rows of 16 bytes in 3 windows (one window holds more than
    2^30 rows): checked by properties that hold at any size -- window counts
    equal a histogram of the timestamps, every entry's row is in its window
    with its key, and rids ascend inside each window (stable)."""
    n = (1 << 30) + 4097
    W = 1 << 20
    say("partition n=2^30+4097")
    i = torch.arange(n, dtype=torch.int64, device="cuda")
    ts = torch.where(i < (1 << 30) + 100, torch.zeros_like(i), (i % 3) * W) + (i % W)
    rows = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    rows[:, 0] = i * -7046029254386353131           # the golden-ratio multiplier as int64
    rows[:, 1] = (ts << 32) | 7
    del i
    keys, rids, off, oob = K.kpa_partition_windows(rows, LAYOUT16, W, 3)
    torch.cuda.synchronize()
    tsr = (rows[:, 1] >> 32) & 0xFFFFFFFF
    cnt = torch.bincount(tsr // W, minlength=3)
    offs = off.cpu().tolist()
    assert offs == [0, int(cnt[0]), int(cnt[0] + cnt[1]), n] and int(oob.item()) == 0
    assert int(cnt[0]) > (1 << 30)
    r = rids.long()
    assert torch.equal(keys, rows[r, 0])
    wt = tsr[r] // W
    for w in range(3):
        a, b = offs[w], offs[w + 1]
        assert bool((wt[a:b] == w).all())
        assert bool((r[a + 1:b] > r[a:b - 1]).all())


def test_sort_segment_of_2_30_entries_is_copied_and_counted(K):
    """A sort segment of 2^30 entries exceeds the look-back words: it comes out
    unchanged and kpa_sort_stats.unsupported_entries reports it; a small
    segment beside it is sorted."""
    big, small = 1 << 30, 5000
    n = big + small
    say("sort segment of 2^30 entries")
    keys = torch.randint(0, 1 << 62, (n,), dtype=torch.int64, device="cuda")
    rids = torch.arange(n, dtype=torch.int32, device="cuda")
    off = dev_u64([0, big, n])
    st = K.new_sort_stats("cuda")
    ok, orr = K.kpa_sort_segmented(keys, rids, off, stats=st)
    torch.cuda.synchronize()
    assert int(st[6].item()) == big
    assert torch.equal(ok[:big], keys[:big]) and torch.equal(orr[:big], rids[:big])
    sk, idx = torch.sort(keys[big:], stable=True)
    assert torch.equal(ok[big:], sk) and torch.equal(orr[big:].long(), idx + big)


@pytest.mark.parametrize("n,n_camps", [(300_001, 100), (70_000, 2000)])
def test_ad_pipeline_counts_views_per_campaign_and_window(K, n, n_camps):
    """The pipeline example of Sec. 4.3 (Select on the event type, KeyUpdate
    ad -> campaign from a sorted table, write-back, KeySwap to time,
    Partition, KeySwap to the campaign, sort, count) against its definition
    counted directly on the host: per tumbling window, the number of view
    events of each campaign (ads missing from the table keep their ad key).
    The table of 2000 campaigns (20000 ads) is searched in device memory,
    the one of 100 campaigns on chip."""
    from paper_1901_01328_amd.pipeline import AdPipeline
    W, n_win = 10 ** 9, 9                       # the last of 10 s of events lies outside
    rows = datagen.gen_ysb(n, seed=n_camps, device="cuda", n_camps=n_camps, ads_per_camp=10)
    rows_h = rows.cpu().numpy().view(np.uint64).copy()
    tk, tv = datagen.ysb_tables(n_camps, 10, seed=n_camps, device="cuda")
    pipe = AdPipeline(n, tk, tv, W, n_win)
    say(f"ad pipeline n={n} campaigns={n_camps}")
    info = pipe.step(rows)
    torch.cuda.synchronize()
    # the definition, counted on the host
    table = dict(zip(tk.cpu().numpy().view(np.uint64).tolist(),
                     tv.cpu().numpy().view(np.uint64).tolist()))
    keep = rows_h[:, 1] == np.uint64(datagen.YSB_VIEW)
    ads, ts = rows_h[keep, 0], rows_h[keep, 2]
    camp = np.array([table.get(int(a), int(a)) for a in ads.tolist()], np.uint64)
    win = ts // np.uint64(W)
    inw = win < np.uint64(n_win)
    assert info["survivors"] == int(keep.sum()) and info["in_windows"] == int(inw.sum())
    missing = sum(1 for a in ads.tolist() if int(a) not in table)
    assert int(pipe.missing.item()) == missing
    gs = u64(pipe.gseg)
    for w in range(n_win):
        ks, cs = np.unique(camp[inw & (win == np.uint64(w))], return_counts=True)
        g0, g1 = int(gs[w]), int(gs[w + 1])
        assert np.array_equal(u64(pipe.gkey)[g0:g1], ks), w
        assert np.array_equal(u64(pipe.gcnt)[g0:g1], cs.astype(np.uint64)), w
    # write-back: kept rows hold their campaign, the others are untouched
    after = rows.cpu().numpy().view(np.uint64)
    assert np.array_equal(after[keep, 3], camp)
    assert np.array_equal(after[~keep, 3], rows_h[~keep, 3])
