"""GPU parity: extract, window partition, radix sort, keyed reduction, top-k and
materialize through the C ABI, element by element against the CPU oracle."""
import numpy as np
import pytest
import torch

import datagen
from datagen.rows import LAYOUT16, LAYOUT32
from gpu_util import dev_u32, dev_u64, kpa_mod, need_gpu, say, u32, u64

pytestmark = pytest.mark.gpu

SIZES = [0, 1, 5, 4095, 4096, 4097, 3 * 4096 + 123, 70001, 262144 + 77]


@pytest.fixture(scope="module")
def K():
    need_gpu()
    return kpa_mod()


def c2_rows(n, seed=11, n_keys=5000, span=10 ** 6):
    return datagen.gen_c2(n, seed=seed, n_keys=n_keys, span_ns=span)


@pytest.mark.parametrize("n", [1, 4097, 70001])
def test_extract(K, orc, n):
    rows = c2_rows(n)
    say(f"extract n={n}")
    k, r = K.kpa_extract(rows.cuda(), LAYOUT32, rid_base=7)
    torch.cuda.synchronize()
    ek, er = orc.extract(rows, LAYOUT32, rid_base=7)
    assert np.array_equal(u64(k), ek) and np.array_equal(u32(r), er)


@pytest.mark.parametrize("layout", ["16", "32"])
def test_extract_value_column(K, layout):
    n = 9001
    if layout == "32":
        rows, lay = c2_rows(n), LAYOUT32
        expect = rows[:, 1].numpy().view(np.uint64)
    else:
        rows, lay = datagen.gen_c1(n, seed=3), LAYOUT16
        expect = rows.numpy().view(np.uint32).reshape(n, 4)[:, 2].astype(np.uint64)
    vals = torch.empty(n, dtype=torch.int64, device="cuda")
    k, r = K.kpa_extract(rows.cuda(), lay, out_vals=vals)
    torch.cuda.synchronize()
    assert np.array_equal(u64(vals), expect)


@pytest.mark.parametrize("n", SIZES)
def test_partition_c2_layout(K, orc, n):
    rows = c2_rows(n, span=10 ** 6)
    W, nw = 10 ** 5, 10
    say(f"partition32 n={n}")
    keys, rids, off, oob = K.kpa_partition_windows(rows.cuda(), LAYOUT32, W, nw)
    torch.cuda.synchronize()
    ek, er, eoff, eoob = orc.partition(rows, LAYOUT32, W, nw)
    assert int(oob.item()) == eoob
    assert np.array_equal(u64(off), eoff)
    m = int(eoff[-1])
    assert np.array_equal(u64(keys)[:m], ek) and np.array_equal(u32(rids)[:m], er)


@pytest.mark.parametrize("n", [4096 * 5 + 1, 100003])
def test_partition_with_out_of_range_and_boundaries(K, orc, n):
    rows = c2_rows(n, span=10 ** 6)
    rows[::97, 2] = 0                    # before origin
    rows[::89, 2] = 10 ** 9              # after the last window
    rows[::13, 2] = 300000 + (torch.arange(rows[::13].shape[0]) % 3) * 100000  # on window edges
    W, nw, origin = 10 ** 5, 7, 12345
    say(f"partition oob n={n}")
    keys, rids, off, oob = K.kpa_partition_windows(rows.cuda(), LAYOUT32, W, nw, win_origin=origin,
                                                   rid_base=3)
    torch.cuda.synchronize()
    ek, er, eoff, eoob = orc.partition(rows, LAYOUT32, W, nw, origin=origin, rid_base=3)
    assert eoob > 0 and int(oob.item()) == eoob
    assert np.array_equal(u64(off), eoff)
    m = int(eoff[-1])
    assert np.array_equal(u64(keys)[:m], ek) and np.array_equal(u32(rids)[:m], er)


def test_partition_256_windows_every_edge(K, orc):
    """256 windows of 1000 ns: timestamps on every window start, one before and
    one after it, and random ones (the window of a timestamp is estimated in
    single precision and corrected against the window starts)."""
    W, nw, origin = 1000, 256, 77
    edges = origin + np.arange(nw + 1, dtype=np.int64) * W
    ts = np.concatenate([edges - 1, edges, edges + 1,
                         origin + np.random.default_rng(5).integers(0, nw * W, 60000)])
    n = len(ts)
    rows = c2_rows(n, span=10 ** 6)
    rows[:, 2] = torch.from_numpy(ts)
    say(f"partition 256 windows n={n}")
    keys, rids, off, oob = K.kpa_partition_windows(rows.cuda(), LAYOUT32, W, nw, win_origin=origin)
    torch.cuda.synchronize()
    ek, er, eoff, eoob = orc.partition(rows, LAYOUT32, W, nw, origin=origin)
    assert int(oob.item()) == eoob == 3   # origin - 1, and the end of the last window and one after
    assert np.array_equal(u64(off), eoff)
    m = int(eoff[-1])
    assert np.array_equal(u64(keys)[:m], ek) and np.array_equal(u32(rids)[:m], er)


def test_partition_16byte_rows_and_huge_window_len(K, orc):
    rows = datagen.gen_c1(50000, seed=3)
    say("partition16")
    keys, rids, off, oob = K.kpa_partition_windows(rows.cuda(), LAYOUT16, 250, 4)
    torch.cuda.synchronize()
    ek, er, eoff, eoob = orc.partition(rows, LAYOUT16, 250, 4)
    assert np.array_equal(u64(off), eoff) and int(oob.item()) == eoob
    m = int(eoff[-1])
    assert np.array_equal(u64(keys)[:m], ek) and np.array_equal(u32(rids)[:m], er)
    # a window length so large that n_win*win_len overflows: exact division path
    big = (1 << 63) + 5
    keys, rids, off, oob = K.kpa_partition_windows(rows.cuda(), LAYOUT16, big, 256)
    torch.cuda.synchronize()
    assert u64(off).tolist()[:2] == [0, 50000] and int(oob.item()) == 0


def key_dist(name, n, rng):
    if name == "uniform64":
        return rng.integers(0, 1 << 63, size=n, dtype=np.uint64) * np.uint64(2) + \
            rng.integers(0, 2, size=n, dtype=np.uint64)
    if name == "small_range":      # high digits constant: passes skipped
        return np.uint64(0xABCD000000000000) + rng.integers(0, 1 << 20, size=n, dtype=np.uint64)
    if name == "few_distinct":
        pool = rng.integers(0, 1 << 63, size=7, dtype=np.uint64)
        return pool[rng.integers(0, 7, size=n)]
    if name == "all_equal":
        return np.full(n, 0xFFFFFFFFFFFFFFFF, dtype=np.uint64)
    if name == "extremes":
        return rng.choice(np.array([0, 1, (1 << 63), (1 << 64) - 1], dtype=np.uint64), size=n)
    if name == "sorted":
        return np.sort(rng.integers(0, 1 << 40, size=n, dtype=np.uint64))
    if name == "reversed":
        return np.sort(rng.integers(0, 1 << 40, size=n, dtype=np.uint64))[::-1].copy()
    raise ValueError(name)


DISTS = ["uniform64", "small_range", "few_distinct", "all_equal", "extremes", "sorted", "reversed"]


@pytest.mark.parametrize("dist", DISTS)
@pytest.mark.parametrize("n", [1, 4096, 4097, 50000, 300007])
def test_radix_sort_single(K, orc, dist, n):
    rng = np.random.default_rng(hash((dist, n)) % (1 << 32))
    keys = key_dist(dist, n, rng)
    rids = rng.permutation(n).astype(np.uint32)
    say(f"sort {dist} n={n}")
    ok, orr = K.kpa_sort(dev_u64(keys), dev_u32(rids))
    torch.cuda.synchronize()
    ek, er = orc.sort(keys, rids)
    assert np.array_equal(u64(ok), ek)
    assert np.array_equal(u32(orr), er)


@pytest.mark.parametrize("dist", ["uniform64", "small_range", "few_distinct"])
def test_radix_sort_segmented(K, orc, dist):
    rng = np.random.default_rng(5)
    sizes = [0, 1, 4096, 0, 4095, 9000, 3, 70001, 0, 128, 40000]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    n = int(off[-1])
    keys = key_dist(dist, n, rng)
    if dist == "small_range":   # a constant segment and a segment with one varying digit
        keys[off[2]:off[3]] = 77
        keys[off[5]:off[6]] = np.uint64(5 << 40) + rng.integers(0, 256, size=sizes[5],
                                                                dtype=np.uint64)
    rids = np.arange(n, dtype=np.uint32)
    say(f"sort segmented {dist}")
    ok, orr = K.kpa_sort_segmented(dev_u64(keys), dev_u32(rids), dev_u64(off), n_cap=n + 1000)
    torch.cuda.synchronize()
    ek, er = orc.sort_segmented(keys, rids, off)
    assert np.array_equal(u64(ok), ek) and np.array_equal(u32(orr), er)


def reduce_expect(orc, keys, rids, off, rows, layout):
    gk, gc, gs, gm, goff = [], [], [], [], [0]
    for a, b in zip(off[:-1], off[1:]):
        a, b = int(a), int(b)
        k, c, s, m = orc.reduce_by_key(keys[a:b], rids[a:b], rows, layout)
        gk.append(k); gc.append(c); gs.append(s); gm.append(m)
        goff.append(goff[-1] + len(k))
    cat = lambda xs: np.concatenate(xs) if xs else np.zeros(0, np.uint64)  # noqa: E731
    return cat(gk), cat(gc), cat(gs), cat(gm), np.array(goff, np.uint64)


@pytest.mark.parametrize("n_keys", [1, 3, 700, 100000])
def test_reduce_by_key_after_sort(K, orc, n_keys):
    n = 150001
    rows = c2_rows(n, seed=21, n_keys=n_keys, span=10 ** 6)
    W, nw = 10 ** 5, 10
    say(f"reduce n_keys={n_keys}")
    d = rows.cuda()
    keys, rids, off, oob = K.kpa_partition_windows(d, LAYOUT32, W, nw)
    sk, sr = K.kpa_sort_segmented(keys, rids, off, n_cap=n)
    gkey, outs, gseg = K.kpa_reduce_by_key(sk, sr, off, d, LAYOUT32, n_cap=n,
                                           want=("cnt", "sum", "max", "gstart"))
    torch.cuda.synchronize()
    hk, hr, hoff, _ = orc.partition(rows, LAYOUT32, W, nw)
    esk, esr = orc.sort_segmented(hk, hr, hoff)
    ek, ec, es, em, eoff = reduce_expect(orc, esk, esr, hoff, rows, LAYOUT32)
    assert np.array_equal(u64(gseg), eoff)
    g = int(eoff[-1])
    assert np.array_equal(u64(gkey)[:g], ek)
    assert np.array_equal(u64(outs["cnt"])[:g], ec)
    assert np.array_equal(u64(outs["sum"])[:g], es)
    assert np.array_equal(u64(outs["max"])[:g], em)
    # gstart: index of each group's first entry = exclusive scan of counts within segments
    starts = []
    for s in range(nw):
        a, b = int(eoff[s]), int(eoff[s + 1])
        starts.append(int(hoff[s]) + np.concatenate([[0], np.cumsum(ec[a:b])[:-1]]) if b > a else [])
    assert np.array_equal(u64(outs["gstart"])[:g], np.concatenate(starts).astype(np.uint64))


def test_reduce_wraps_and_u32_values(K, orc):
    n = 9000
    rows = c2_rows(n, seed=4, n_keys=3)
    rows[:, 1] = -1  # value 2^64-1 everywhere: sums wrap
    d = rows.cuda()
    keys, rids = K.kpa_extract(d, LAYOUT32)
    off = dev_u64([0, n])
    sk, sr = K.kpa_sort_segmented(keys, rids, off)
    gkey, outs, gseg = K.kpa_reduce_by_key(sk, sr, off, d, LAYOUT32)
    torch.cuda.synchronize()
    esk, esr = orc.sort(u64(keys), u32(rids))
    ek, ec, es, em = orc.reduce_by_key(esk, esr, rows, LAYOUT32)
    g = len(ek)
    assert np.array_equal(u64(outs["sum"])[:g], es) and np.array_equal(u64(outs["max"])[:g], em)
    rows16 = datagen.gen_c1(20000, seed=8)
    rows16[:, 1] |= 0xFFFFFFFF  # u32 value 2^32-1
    d16 = rows16.cuda()
    keys, rids = K.kpa_extract(d16, LAYOUT16)
    off = dev_u64([0, 20000])
    sk, sr = K.kpa_sort_segmented(keys, rids, off)
    gkey, outs, gseg = K.kpa_reduce_by_key(sk, sr, off, d16, LAYOUT16)
    torch.cuda.synchronize()
    esk, esr = orc.sort(u64(keys), u32(rids))
    ek, ec, es, em = orc.reduce_by_key(esk, esr, rows16, LAYOUT16)
    g = len(ek)
    assert np.array_equal(u64(outs["sum"])[:g], es) and np.array_equal(u64(outs["cnt"])[:g], ec)


@pytest.mark.parametrize("n_keys", [5, 3000, 200000])
def test_topk_by_sum(K, orc, n_keys):
    n = 200000
    rows = c2_rows(n, seed=31, n_keys=n_keys)
    rows[::5, 1] = 7   # many equal sums for the tie order
    W, nw = 10 ** 5, 10
    d = rows.cuda()
    say(f"topk n_keys={n_keys}")
    keys, rids, off, oob = K.kpa_partition_windows(d, LAYOUT32, W, nw)
    sk, sr = K.kpa_sort_segmented(keys, rids, off, n_cap=n)
    gkey, outs, gseg = K.kpa_reduce_by_key(sk, sr, off, d, LAYOUT32, n_cap=n, want=("sum",))
    tk, ts, tn = K.kpa_topk_by_sum(gkey, outs["sum"], gseg, k=10, g_cap=n)
    torch.cuda.synchronize()
    hk, hr, hoff, _ = orc.partition(rows, LAYOUT32, W, nw)
    esk, esr = orc.sort_segmented(hk, hr, hoff)
    ek, ec, es, em, eoff = reduce_expect(orc, esk, esr, hoff, rows, LAYOUT32)
    tk, ts, tn = u64(tk).reshape(nw, 10), u64(ts).reshape(nw, 10), u32(tn)
    for w in range(nw):
        a, b = int(eoff[w]), int(eoff[w + 1])
        xk, xs = orc.topk_by_sum(ek[a:b], es[a:b], 10)
        assert tn[w] == len(xk)
        assert np.array_equal(tk[w][:len(xk)], xk) and np.array_equal(ts[w][:len(xs)], xs)


@pytest.mark.parametrize("layout,n", [(LAYOUT32, 70001), (LAYOUT16, 4097)])
def test_materialize(K, orc, layout, n):
    rows = c2_rows(n) if layout is LAYOUT32 else datagen.gen_c1(n)
    rng = np.random.default_rng(1)
    rids = rng.integers(0, n, size=n // 2 + 3).astype(np.uint32)
    say(f"materialize {layout.row_bytes} n={n}")
    out = K.kpa_materialize(dev_u32(rids), rows.cuda(), layout.row_bytes)
    torch.cuda.synchronize()
    exp = orc.materialize(rids, rows, layout)
    got = out.cpu().numpy().view(np.uint8)[:exp.size]
    assert np.array_equal(got, exp)


def test_c1_end_to_end(K, orc):
    """The small plain workload: 2^20 16-byte rows, 1000 keys, one 1 s window."""
    n = 1 << 20
    rows = datagen.gen_c1(n, seed=1)
    d = rows.cuda()
    say("c1 end to end")
    keys, rids, off, oob = K.kpa_partition_windows(d, LAYOUT16, 1000, 1)
    sk, sr = K.kpa_sort_segmented(keys, rids, off, n_cap=n)
    gkey, outs, gseg = K.kpa_reduce_by_key(sk, sr, off, d, LAYOUT16, n_cap=n, want=("cnt", "sum"))
    torch.cuda.synchronize()
    g, tk, ts, cs = orc.window_aggregate(rows, LAYOUT16, 1000, 1, k=10)
    hk, hr, hoff, hoob = orc.partition(rows, LAYOUT16, 1000, 1)
    ek, ec, es, em = orc.reduce_by_key(hk, hr, rows, LAYOUT16)
    assert int(oob.item()) == 0 and len(ek) == 1000 == int(g[0])
    assert u64(gseg).tolist() == [0, 1000]
    assert np.array_equal(u64(gkey)[:1000], ek)
    assert np.array_equal(u64(outs["cnt"])[:1000], ec)
    assert np.array_equal(u64(outs["sum"])[:1000], es)


def test_reduce_from_staged_value_column(K, orc):
    """Partition stages the value column; the reduction reading it as 8-byte rows
    equals the oracle reading full rows."""
    from paper_1901_01328_amd.pipeline import VALUE_COLUMN
    n = 123457
    rows = c2_rows(n, seed=41, n_keys=20)   # long runs crossing many tiles
    W, nw = 10 ** 5, 10
    d = rows.cuda()
    vals = torch.empty(n, dtype=torch.int64, device="cuda")
    say("reduce from staged values")
    keys, rids, off, oob = K.kpa_partition_windows(d, LAYOUT32, W, nw, out_vals=vals)
    sk, sr = K.kpa_sort_segmented(keys, rids, off, n_cap=n)
    gkey, outs, gseg = K.kpa_reduce_by_key(sk, sr, off, vals, VALUE_COLUMN, n_cap=n,
                                           want=("cnt", "sum", "max", "gstart"))
    torch.cuda.synchronize()
    assert np.array_equal(u64(vals), u64(rows[:, 1].contiguous()))
    hk, hr, hoff, _ = orc.partition(rows, LAYOUT32, W, nw)
    esk, esr = orc.sort_segmented(hk, hr, hoff)
    ek, ec, es, em, eoff = reduce_expect(orc, esk, esr, hoff, rows, LAYOUT32)
    g = int(eoff[-1])
    assert np.array_equal(u64(gseg), eoff)
    assert np.array_equal(u64(gkey)[:g], ek)
    assert np.array_equal(u64(outs["cnt"])[:g], ec)
    assert np.array_equal(u64(outs["sum"])[:g], es)
    assert np.array_equal(u64(outs["max"])[:g], em)


def test_pipeline_twice_same_result(K, orc):
    """Run-to-run equality of the whole windowed step (race canary)."""
    from paper_1901_01328_amd.pipeline import WindowAggregation
    n = 300001
    rows = c2_rows(n, seed=42, n_keys=3000)
    d = rows.cuda()
    p = WindowAggregation(n, LAYOUT32, 10 ** 5, 10, device="cuda")
    p.step(d)
    torch.cuda.synchronize()
    g = int(p.gseg[-1].item())
    first = [p.skeys.clone(), p.srids.clone()] + [t[:g].clone() for t in
                                                 (p.gkey, p.g["sum"], p.g["max"])]
    first.append(p.top_key.clone())
    p.step(d)
    torch.cuda.synchronize()
    second = [p.skeys, p.srids] + [t[:g] for t in (p.gkey, p.g["sum"], p.g["max"])]
    second.append(p.top_key)
    assert int(p.gseg[-1].item()) == g
    for a, b in zip(first, second):
        assert torch.equal(a, b)


@pytest.mark.parametrize("algo", ["learned", "radix"])
def test_window_pipeline_routes_match_oracle(K, orc, algo):
    """The windowed pipeline over three batches (the learned route's models
    come from the previous batch's windows; its first batch sorts by radix):
    the sorted window KPAs and per-window count/sum/max per key against the
    oracle after every batch."""
    from paper_1901_01328_amd.pipeline import WindowAggregation
    n, W, nw = 400001, 10 ** 5, 10
    a = K.KPA_SORT_LEARNED if algo == "learned" else K.KPA_SORT_RADIX
    p = WindowAggregation(n, LAYOUT32, W, nw, algo=a, device="cuda")
    for batch in range(3):
        rows = c2_rows(n, seed=60 + batch, n_keys=20000)
        say(f"window pipeline {algo} batch {batch}")
        p.step(rows.cuda())
        torch.cuda.synchronize()
        hk, hr, hoff, _ = orc.partition(rows, LAYOUT32, W, nw)
        gseg = u64(p.gseg)
        for w in range(nw):
            a0, b0 = int(hoff[w]), int(hoff[w + 1])
            sk, sr = orc.sort(hk[a0:b0], hr[a0:b0])
            assert np.array_equal(u64(p.skeys)[a0:b0], sk) and np.array_equal(
                u32(p.srids)[a0:b0], sr), (batch, w)
            ek, ec, es, em = orc.reduce_by_key(sk, sr, rows, LAYOUT32)
            g0, g1 = int(gseg[w]), int(gseg[w + 1])
            assert g1 - g0 == len(ek), (batch, w)
            assert np.array_equal(u64(p.gkey)[g0:g1], ek), (batch, w)
            assert np.array_equal(u64(p.g["cnt"])[g0:g1], ec), (batch, w)
            assert np.array_equal(u64(p.g["sum"])[g0:g1], es), (batch, w)
            assert np.array_equal(u64(p.g["max"])[g0:g1], em), (batch, w)
