"""GPU parity: merge, multiway merge, join (count, sum of products, pairs) and
median per key, element by element against the CPU oracle."""
import numpy as np
import pytest
import torch

import datagen
from datagen.rows import LAYOUT16, LAYOUT32
from gpu_util import dev_u32, dev_u64, kpa_mod, need_gpu, say, u32, u64

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    need_gpu()
    return kpa_mod()


def sorted_kpa(orc, rng, n, pool_size, rid0=0):
    pool = rng.integers(0, 1 << 63, size=max(pool_size, 1), dtype=np.uint64) * np.uint64(2)
    keys = pool[rng.integers(0, len(pool), size=n)]
    rids = np.arange(rid0, rid0 + n, dtype=np.uint32)
    return orc.sort(keys, rids)


@pytest.mark.parametrize("na,nb", [(0, 5), (7, 0), (1, 1), (4096, 4096), (5000, 123),
                                   (100003, 77777), (300000, 1)])
def test_merge(K, orc, na, nb):
    rng = np.random.default_rng(na * 7 + nb)
    pool = 50 if na + nb > 1000 else 5     # many equal keys across A and B
    ak, ar = sorted_kpa(orc, rng, na, pool, 0)
    bk, br = sorted_kpa(orc, rng, nb, pool, na)
    say(f"merge {na}+{nb}")
    ok, orr = K.kpa_merge(dev_u64(ak), dev_u32(ar), dev_u64(bk), dev_u32(br))
    torch.cuda.synchronize()
    ek, er = orc.merge(ak, ar, bk, br)
    assert np.array_equal(u64(ok)[:na + nb], ek) and np.array_equal(u32(orr)[:na + nb], er)


MANY_RUNS = [int(x) for x in np.random.default_rng(11).integers(0, 9000, 300)]


# Up to 1024 nonempty runs every round is one launch pair over all its pairs;
# 1100 runs take the per-pair launches.  lead: entries before the first run
# (run_off[0] > 0).
@pytest.mark.parametrize("sizes,lead", [([10], 0), ([3, 0, 9], 0), ([4096] * 7, 0),
                                        ([0, 50000, 1, 0, 7777, 30000, 2], 0), ([1000] * 16, 0),
                                        ([5000, 4096, 4097, 1, 8191, 8193, 0, 12288], 13),
                                        (MANY_RUNS, 0), ([1] * 300, 5), ([3] * 1100, 0),
                                        ([0, 0, 6000, 0], 7)])
def test_merge_runs(K, orc, sizes, lead):
    rng = np.random.default_rng(len(sizes) + lead)
    ks, rs = [rng.integers(0, 1 << 63, lead, dtype=np.uint64)], [np.zeros(lead, np.uint32)]
    base = 0
    for s in sizes:
        k, r = sorted_kpa(orc, rng, s, 200, base)
        ks.append(k)
        rs.append(r)
        base += s
    keys = np.concatenate(ks)
    rids = np.concatenate(rs)
    off = (lead + np.concatenate([[0], np.cumsum(sizes)])).astype(np.uint64)
    say(f"merge_runs {len(sizes)} runs, {base} entries, lead {lead}")
    ok, orr = K.kpa_merge_runs(dev_u64(keys), dev_u32(rids), off.tolist())
    torch.cuda.synchronize()
    ek, er = orc.sort(keys[lead:], rids[lead:])   # stable: equal keys keep run order
    n = base
    assert np.array_equal(u64(ok)[:n], ek) and np.array_equal(u32(orr)[:n], er)


def windows(K, rows, layout, W, nw):
    keys, rids, off, oob = K.kpa_partition_windows(rows, layout, W, nw)
    sk, sr = K.kpa_sort_segmented(keys, rids, off, n_cap=keys.numel())
    return sk, sr, off


def c3_rows(n, side, n_keys, seed=3, span=10 ** 6):
    return datagen.gen_c3(n, seed=seed, side=side, n_keys=n_keys, span_ns=span)


@pytest.mark.parametrize("n,n_keys", [(1, 3), (5000, 1 << 20), (70001, 30000), (200000, 1 << 24),
                                      (40000, 7)])
def test_join_count_sumprod(K, orc, n, n_keys):
    W, nw = 10 ** 5, 10
    L = c3_rows(n, 0, n_keys)
    R = c3_rows(n + 17, 1, n_keys)
    dl, dr = L.cuda(), R.cuda()
    lk, lr, loff = windows(K, dl, LAYOUT32, W, nw)
    rk, rr, roff = windows(K, dr, LAYOUT32, W, nw)
    say(f"join n={n} keys={n_keys}")
    cnt, sp, _, npairs = K.kpa_join(lk, lr, loff, rk, rr, roff, dl, dr, LAYOUT32)
    torch.cuda.synchronize()
    hl = orc.partition(L, LAYOUT32, W, nw)
    hr = orc.partition(R, LAYOUT32, W, nw)
    tot = 0
    for w in range(nw):
        a0, a1 = int(hl[2][w]), int(hl[2][w + 1])
        b0, b1 = int(hr[2][w]), int(hr[2][w + 1])
        ec, es, _, enp = orc.join(hl[0][a0:a1], hl[1][a0:a1], hr[0][b0:b1], hr[1][b0:b1], L, R,
                                  LAYOUT32)
        assert int(u64(cnt)[w]) == ec and int(u64(sp)[w]) == es
        tot += ec
    assert int(u64(npairs)[0]) == tot


def test_join_pairs_with_heavy_key_and_capacity(K, orc):
    W, nw = 10 ** 5, 4
    n = 20000
    L = c3_rows(n, 0, 500)
    R = c3_rows(n, 1, 500)
    L[::3, 0] = R[0, 0]          # one key heavy on both sides
    R[::5, 0] = R[0, 0]
    dl, dr = L.cuda(), R.cuda()
    lk, lr, loff = windows(K, dl, LAYOUT32, W, nw)
    rk, rr, roff = windows(K, dr, LAYOUT32, W, nw)
    hl = orc.partition(L, LAYOUT32, W, nw)
    hr = orc.partition(R, LAYOUT32, W, nw)
    exp_pairs, exp_cnt = [], []
    for w in range(nw):
        a0, a1 = int(hl[2][w]), int(hl[2][w + 1])
        b0, b1 = int(hr[2][w]), int(hr[2][w + 1])
        ec, es, pairs, enp = orc.join(hl[0][a0:a1], hl[1][a0:a1], hr[0][b0:b1], hr[1][b0:b1], L, R,
                                      LAYOUT32, pairs_cap=10 ** 7)
        exp_pairs.append(pairs)
        exp_cnt.append(ec)
    exp = np.concatenate(exp_pairs)
    total = len(exp)
    say(f"join pairs total={total}")
    cnt, sp, pairs, npairs = K.kpa_join(lk, lr, loff, rk, rr, roff, dl, dr, LAYOUT32,
                                        pairs_cap=total + 5)
    torch.cuda.synchronize()
    assert int(u64(npairs)[0]) == total == sum(exp_cnt)
    assert np.array_equal(u64(pairs)[:total], exp)
    # a capacity below the total: the first `cap` pairs are written, the total reported
    cap = total // 3
    cnt, sp, pairs, npairs = K.kpa_join(lk, lr, loff, rk, rr, roff, dl, dr, LAYOUT32,
                                        pairs_cap=cap)
    torch.cuda.synchronize()
    assert int(u64(npairs)[0]) == total
    assert np.array_equal(u64(pairs)[:cap], exp[:cap])


def test_join_no_match_and_empty_windows(K, orc):
    W, nw = 10 ** 5, 6
    L = c3_rows(3000, 0, 1 << 24, seed=1, span=3 * 10 ** 5)   # windows 3..5 empty
    R = c3_rows(3000, 1, 1 << 24, seed=2, span=3 * 10 ** 5)
    L[:, 0] |= 1     # odd keys on the left,
    R[:, 0] &= ~1    # even keys on the right: no match anywhere
    dl, dr = L.cuda(), R.cuda()
    lk, lr, loff = windows(K, dl, LAYOUT32, W, nw)
    rk, rr, roff = windows(K, dr, LAYOUT32, W, nw)
    cnt, sp, _, npairs = K.kpa_join(lk, lr, loff, rk, rr, roff, dl, dr, LAYOUT32)
    torch.cuda.synchronize()
    assert u64(cnt).tolist() == [0] * nw and u64(sp).tolist() == [0] * nw
    assert int(u64(npairs)[0]) == 0


@pytest.mark.parametrize("n,n_keys,span", [(5000, 1 << 20, None), (70001, 30000, None),
                                           (200000, 1 << 24, None), (40000, 7, None),
                                           (3000, 1 << 24, 3 * 10 ** 5)])
def test_join_runs_equals_join(K, orc, n, n_keys, span):
    """The join of two run lists (each key's count and sum, from the median
    pass) equals the join of the sorted KPAs and the oracle, window by
    window; the last case leaves windows 3..9 empty on both sides."""
    W, nw = 10 ** 5, 10
    kw = {} if span is None else {"span": span}
    L = c3_rows(n, 0, n_keys, **kw)
    R = c3_rows(n + 17, 1, n_keys, **kw)
    dl, dr = L.cuda(), R.cuda()
    lk, lr, loff = windows(K, dl, LAYOUT32, W, nw)
    rk, rr, roff = windows(K, dr, LAYOUT32, W, nw)
    say(f"join runs n={n} keys={n_keys}")
    runs = []
    for k_, r_, o_, d_ in ((lk, lr, loff, dl), (rk, rr, roff, dr)):
        o = {"cnt": torch.empty(k_.numel(), dtype=torch.int64, device="cuda"),
             "sum": torch.empty(k_.numel(), dtype=torch.int64, device="cuda")}
        gk, _, gseg = K.kpa_median_by_key(k_, r_, o_, d_, LAYOUT32, outs=o)
        runs.append((gk, o["cnt"], o["sum"], gseg))
    (a, b, c, d), (e, f, g, h) = runs
    cnt, sp = K.kpa_join_runs(a, b, c, d, e, f, g, h)
    cnt2, sp2, _, _ = K.kpa_join(lk, lr, loff, rk, rr, roff, dl, dr, LAYOUT32)
    torch.cuda.synchronize()
    assert np.array_equal(u64(cnt), u64(cnt2)) and np.array_equal(u64(sp), u64(sp2))
    hl = orc.partition(L, LAYOUT32, W, nw)
    hr = orc.partition(R, LAYOUT32, W, nw)
    for w in range(nw):
        a0, a1 = int(hl[2][w]), int(hl[2][w + 1])
        b0, b1 = int(hr[2][w]), int(hr[2][w + 1])
        ec, es, _, _ = orc.join(hl[0][a0:a1], hl[1][a0:a1], hr[0][b0:b1], hr[1][b0:b1], L, R,
                                LAYOUT32)
        assert int(u64(cnt)[w]) == ec and int(u64(sp)[w]) == es, w


def test_median_and_sums_at_every_size_class_edge(K, orc):
    """Groups of exactly the sizes where the median changes method (one
    thread up to 16 values, one workgroup in LDS up to 4096, radix selection
    above), with values that wrap the 64-bit sum: medians, counts and sums
    against the oracle.  Keys interleave in arrival order, so every group is
    spread over the window."""
    sizes = [1, 2, 15, 16, 17, 18, 255, 4095, 4096, 4097, 9001]
    rng = np.random.default_rng(41)
    keys = np.repeat(rng.integers(1, 2 ** 63, len(sizes), dtype=np.int64), sizes)
    rng.shuffle(keys)
    n = len(keys)
    rows = torch.zeros((n, 4), dtype=torch.int64)
    rows[:, 0] = torch.from_numpy(keys)
    rows[:, 1] = torch.from_numpy(rng.integers(-2 ** 63, 2 ** 63 - 1, n, dtype=np.int64))
    rows[::7, 1] = 99                   # repeated values
    rows[:, 2] = torch.arange(n) * 10   # one window
    d = rows.cuda()
    sk, sr, off = windows(K, d, LAYOUT32, 10 ** 9, 1)
    say(f"median edges n={n}")
    sums = {"cnt": torch.empty(n, dtype=torch.int64, device="cuda"),
            "sum": torch.empty(n, dtype=torch.int64, device="cuda")}
    gk, gm, gseg = K.kpa_median_by_key(sk, sr, off, d, LAYOUT32, outs=sums)
    torch.cuda.synchronize()
    hk, hr, hoff, _ = orc.partition(rows, LAYOUT32, 10 ** 9, 1)
    sk_, sr_ = orc.sort(hk, hr)
    ek, em = orc.median_by_key(sk_, sr_, rows, LAYOUT32)
    _, ec, es, _ = orc.reduce_by_key(sk_, sr_, rows, LAYOUT32)
    g = len(ek)
    assert g == len(sizes) and int(u64(gseg)[1]) == g
    assert sorted(ec.tolist()) == sorted(sizes)
    assert np.array_equal(u64(gk)[:g], ek) and np.array_equal(u64(gm)[:g], em)
    assert np.array_equal(u64(sums["cnt"])[:g], ec) and np.array_equal(u64(sums["sum"])[:g], es)


def median_expect(orc, keys, rids, off, rows, layout):
    gk, gm, goff = [], [], [0]
    for a, b in zip(off[:-1], off[1:]):
        k, m = orc.median_by_key(keys[int(a):int(b)], rids[int(a):int(b)], rows, layout)
        gk.append(k)
        gm.append(m)
        goff.append(goff[-1] + len(k))
    return np.concatenate(gk), np.concatenate(gm), np.array(goff, np.uint64)


@pytest.mark.parametrize("case", ["uniform", "medium_runs", "big_runs", "u32_values"])
def test_median_by_key(K, orc, case):
    W, nw = 10 ** 5, 10
    if case == "uniform":
        rows, lay = c3_rows(150001, 0, 1 << 17), LAYOUT32
    elif case == "medium_runs":
        rows, lay = c3_rows(150001, 0, 400), LAYOUT32
    elif case == "big_runs":
        rows, lay = c3_rows(150001, 0, 2), LAYOUT32
        rows[::7, 1] = 12345        # repeated values inside big runs
    else:
        rows, lay = datagen.gen_c1(100001, seed=5), LAYOUT16
        W, nw = 100, 10
    d = rows.cuda()
    sk, sr, off = windows(K, d, lay, W, nw)
    say(f"median {case}")
    cap = sk.numel()
    sums = {"cnt": torch.empty(cap, dtype=torch.int64, device="cuda"),
            "sum": torch.empty(cap, dtype=torch.int64, device="cuda")}
    gk, gm, gseg = K.kpa_median_by_key(sk, sr, off, d, lay, outs=sums)
    torch.cuda.synchronize()
    hk, hr, hoff, _ = orc.partition(rows, lay, W, nw)
    ek, em, eoff = median_expect(orc, hk, hr, hoff, rows, lay)
    assert np.array_equal(u64(gseg), eoff)
    g = int(eoff[-1])
    assert np.array_equal(u64(gk)[:g], ek)
    assert np.array_equal(u64(gm)[:g], em)
    # the counts and value sums written on the way equal the keyed reduction's
    ec, es = [], []
    for a, b in zip(hoff[:-1], hoff[1:]):
        _, c, sm, _ = orc.reduce_by_key(hk[int(a):int(b)], hr[int(a):int(b)], rows, lay)
        ec.append(c)
        es.append(sm)
    assert np.array_equal(u64(sums["cnt"])[:g], np.concatenate(ec))
    assert np.array_equal(u64(sums["sum"])[:g], np.concatenate(es))
    # without them the medians are the same
    gk2, gm2, _ = K.kpa_median_by_key(sk, sr, off, d, lay)
    torch.cuda.synchronize()
    assert np.array_equal(u64(gm2)[:g], em) and np.array_equal(u64(gk2)[:g], ek)
