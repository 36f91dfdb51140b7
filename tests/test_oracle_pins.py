"""Pins for the CPU oracle: brute force on tiny inputs, invariants, closed
forms, a hand-worked example and library special cases.  CPU only."""
import json
import os

import numpy as np
import pytest
import torch

import datagen
from datagen.rows import LAYOUT16, LAYOUT32

M64 = (1 << 64) - 1
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def rows16(triples):
    key = torch.tensor([t[0] for t in triples], dtype=torch.int64)
    val = torch.tensor([t[1] for t in triples], dtype=torch.int64)
    ts = torch.tensor([t[2] for t in triples], dtype=torch.int64)
    return datagen.pack_rows16(key, val, ts)


def s64(x):
    x &= M64
    return x - (1 << 64) if x >= (1 << 63) else x


def rows32(quads):
    t = torch.tensor([[s64(v) for v in q] for q in quads], dtype=torch.int64).reshape(-1, 4)
    return t


def rand_rows32(rng, n, n_keys, ts_span, val_bits=64, extreme=False):
    keys = rng.integers(0, 1 << 63, size=max(n_keys, 1), dtype=np.uint64) * np.uint64(2) + \
        rng.integers(0, 2, size=max(n_keys, 1), dtype=np.uint64)
    if extreme:
        keys[0] = 0
        if n_keys > 1:
            keys[1] = np.uint64(M64)
    out = []
    for i in range(n):
        k = int(keys[rng.integers(0, len(keys))])
        v = int(rng.integers(0, 1 << 62)) * 4 + int(rng.integers(0, 4))
        v &= (1 << val_bits) - 1
        if extreme and rng.random() < 0.3:
            v = M64
        ts = int(rng.integers(0, ts_span))
        out.append((k, v, ts, i))
    return out


# ----------------------------------------------------------------- golden ---

def test_golden_tiny_window(orc):
    g = json.load(open(os.path.join(GOLD, "tiny_window.json")))
    rows = rows16(g["rows"])
    lay = LAYOUT16
    e = g["expect"]
    keys, rids, off, oob = orc.partition(rows, lay, g["window_len"], g["n_win"])
    assert oob == e["oob"]
    assert off.tolist() == e["win_off"]
    assert keys.tolist() == e["partition_keys"] and rids.tolist() == e["partition_rids"]
    sk, sr = orc.sort_segmented(keys, rids, off)
    assert sk.tolist() == e["sorted_keys"] and sr.tolist() == e["sorted_rids"]
    for w, name in ((0, "w0_groups"), (1, "w1_groups")):
        a, b = int(off[w]), int(off[w + 1])
        gk, gc, gs, gm = orc.reduce_by_key(sk[a:b], sr[a:b], rows, lay)
        assert gk.tolist() == e[name]["key"]
        assert gc.tolist() == e[name]["cnt"]
        assert gs.tolist() == e[name]["sum"]
        assert gm.tolist() == e[name]["max"]
        mk, mv = orc.median_by_key(sk[a:b], sr[a:b], rows, lay)
        assert mk.tolist() == e[name]["key"] and mv.tolist() == e[name]["median"]
    gk, gc, gs, gm = orc.reduce_by_key(sk[4:7], sr[4:7], rows, lay)
    tk, ts = orc.topk_by_sum(gk, gs, 10)
    assert tk.tolist() == e["w1_top10"]["key"] and ts.tolist() == e["w1_top10"]["sum"]
    cnt, sp, pairs, npairs = orc.join(sk[0:4], sr[0:4], sk[4:7], sr[4:7], rows, rows, lay, 16)
    j = e["join_w0_with_w1"]
    assert cnt == j["count"] and sp == j["sumprod"] and npairs == j["count"]
    assert pairs.tolist() == j["pairs"]
    mat = orc.materialize(sr[0:4], rows, lay)
    raw = rows.numpy().view(np.uint8).reshape(-1, 16)
    assert np.array_equal(mat.reshape(-1, 16), raw[e["materialize_w0_rids"]])


# -------------------------------------------------------------- partition ---

@pytest.mark.parametrize("seed", range(40))
def test_partition_brute_force(orc, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(0, 65))
    W = int(rng.integers(1, 50))
    nw = int(rng.integers(1, 6))
    origin = int(rng.integers(0, 20))
    rows = rand_rows32(rng, n, int(rng.integers(1, 10)), origin + nw * W + 30)
    # timestamps exactly on window edges
    for i in range(0, n, 7):
        k, v, _, p = rows[i]
        rows[i] = (k, v, origin + W * int(rng.integers(0, nw + 1)), p)
    t = rows32(rows)
    keys, rids, off, oob = orc.partition(t, LAYOUT32, W, nw, origin=origin, rid_base=5)
    exp = [[] for _ in range(nw)]
    bad = 0
    for i, (k, v, ts, _) in enumerate(rows):
        if ts < origin or ts >= origin + nw * W:
            bad += 1
            continue
        w = 0
        while not (origin + w * W <= ts < origin + (w + 1) * W):
            w += 1
        exp[w].append((k, i + 5))
    assert oob == bad
    assert int(off[-1]) == n - bad  # conserved count
    for w in range(nw):
        a, b = int(off[w]), int(off[w + 1])
        got = list(zip(keys[a:b].tolist(), rids[a:b].tolist()))
        assert got == exp[w]
        assert all(rids[a:b][i] < rids[a:b][i + 1] for i in range(b - a - 1))


def test_partition_empty(orc):
    t = torch.zeros((0, 4), dtype=torch.int64)
    keys, rids, off, oob = orc.partition(t, LAYOUT32, 10, 3)
    assert keys.size == 0 and off.tolist() == [0, 0, 0, 0] and oob == 0


# ------------------------------------------------------------------- sort ---

def brute_sort(keys, rids):
    n = len(keys)
    out = [None] * n
    for i in range(n):
        pos = sum(1 for j in range(n) if keys[j] < keys[i]) + \
            sum(1 for j in range(i) if keys[j] == keys[i])
        out[pos] = (keys[i], rids[i])
    return out


def key_cases(rng):
    yield np.array([], np.uint64)
    yield np.array([5], np.uint64)
    yield np.full(17, 42, np.uint64)
    yield np.arange(30, dtype=np.uint64)
    yield np.arange(30, dtype=np.uint64)[::-1].copy()
    yield np.array([M64, 0, M64, 1 << 63, 0, (1 << 63) - 1], np.uint64)
    for _ in range(60):
        n = int(rng.integers(1, 65))
        pool = rng.integers(0, 1 << 63, size=int(rng.integers(1, 70)), dtype=np.uint64) * \
            np.uint64(2) + np.uint64(1)
        yield pool[rng.integers(0, len(pool), size=n)]


def test_sort_brute_force_and_invariants(orc):
    rng = np.random.default_rng(7)
    for keys in key_cases(rng):
        n = len(keys)
        rids = rng.permutation(max(n, 1)).astype(np.uint32)[:n]
        sk, sr = orc.sort(keys, rids)
        assert list(zip(sk.tolist(), sr.tolist())) == brute_sort(keys.tolist(), rids.tolist())
        assert all(sk[i] <= sk[i + 1] for i in range(n - 1))            # sorted
        assert sorted(sr.tolist()) == sorted(rids.tolist())               # permutation
        assert sorted(sk.tolist()) == sorted(keys.tolist())               # key multiset
        # library special case: a stable argsort on unsigned keys
        o = np.argsort(keys, kind="stable")
        assert np.array_equal(sk, keys[o]) and np.array_equal(sr, rids[o])


def test_sort_segmented_matches_per_segment(orc):
    rng = np.random.default_rng(3)
    keys = rng.integers(0, 1 << 40, size=300, dtype=np.uint64)
    rids = np.arange(300, dtype=np.uint32)
    off = np.array([0, 0, 17, 17, 150, 299, 300], np.uint64)
    sk, sr = orc.sort_segmented(keys, rids, off)
    for a, b in zip(off[:-1], off[1:]):
        a, b = int(a), int(b)
        ek, er = orc.sort(keys[a:b], rids[a:b])
        assert np.array_equal(sk[a:b], ek) and np.array_equal(sr[a:b], er)


# ------------------------------------------------------------------ merge ---

def test_merge_equals_sort_of_union(orc):
    rng = np.random.default_rng(11)
    for _ in range(50):
        na, nb = int(rng.integers(0, 40)), int(rng.integers(0, 40))
        pool = rng.integers(0, 1 << 63, size=int(rng.integers(1, 20)), dtype=np.uint64)
        ak = pool[rng.integers(0, len(pool), size=na)]
        bk = pool[rng.integers(0, len(pool), size=nb)]
        ar = np.arange(na, dtype=np.uint32)
        br = np.arange(na, na + nb, dtype=np.uint32)
        ak, ar = orc.sort(ak, ar)
        bk, br = orc.sort(bk, br)
        mk, mr = orc.merge(ak, ar, bk, br)
        # stable sort of the concatenation A then B equals the stable merge
        ck, cr = orc.sort(np.concatenate([ak, bk]), np.concatenate([ar, br]))
        assert np.array_equal(mk, ck) and np.array_equal(mr, cr)
        assert list(zip(mk.tolist(), mr.tolist())) == brute_sort(
            np.concatenate([ak, bk]).tolist(), np.concatenate([ar, br]).tolist())


# ----------------------------------------------------------------- reduce ---

@pytest.mark.parametrize("seed", range(30))
def test_reduce_brute_force_and_invariants(orc, seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(0, 65))
    rows = rand_rows32(rng, n, int(rng.integers(1, 12)), 100, extreme=(seed % 3 == 0))
    t = rows32(rows)
    keys, rids = orc.extract(t, LAYOUT32)
    perm = rng.permutation(n)
    keys, rids = keys[perm], rids[perm]             # input order is free
    gk, gc, gs, gm = orc.reduce_by_key(keys, rids, t, LAYOUT32)
    distinct = sorted(set(r[0] for r in rows))
    assert gk.tolist() == distinct                   # G = #distinct, ascending
    for g, k in enumerate(distinct):
        vals = [r[1] for r in rows if r[0] == k]
        assert gc[g] == len(vals)
        assert int(gs[g]) == sum(vals) % (1 << 64)
        assert int(gm[g]) == max(vals)
    assert int(gc.sum()) == n                        # conserved count
    assert int(sum(int(x) for x in gs.tolist())) % (1 << 64) == sum(r[1] for r in rows) % (1 << 64)
    if n:
        assert int(gm.max()) == max(r[1] for r in rows)


def test_reduce_sum_wraps(orc):
    t = rows32([(1, M64, 0, 0), (1, M64, 0, 0), (2, 3, 0, 0)])
    keys, rids = orc.extract(t, LAYOUT32)
    gk, gc, gs, gm = orc.reduce_by_key(keys, rids, t, LAYOUT32)
    assert gk.tolist() == [1, 2] and gc.tolist() == [2, 1]
    assert int(gs[0]) == M64 - 1 and int(gm[0]) == M64


def test_reduce_u32_values(orc):
    t = rows16([(9, 0xFFFFFFFF, 1), (9, 1, 2)])
    keys, rids = orc.extract(t, LAYOUT16)
    gk, gc, gs, gm = orc.reduce_by_key(keys, rids, t, LAYOUT16)
    assert int(gs[0]) == 1 << 32 and int(gm[0]) == 0xFFFFFFFF


# ------------------------------------------------------------------- topk ---

def test_topk_brute_force(orc):
    rng = np.random.default_rng(5)
    for _ in range(50):
        g = int(rng.integers(0, 40))
        gk = rng.permutation(1000)[:g].astype(np.uint64)
        gs = rng.integers(0, 6, size=g).astype(np.uint64)   # many equal sums
        k = int(rng.integers(1, 15))
        tk, ts = orc.topk_by_sum(gk, gs, k)
        exp = sorted(zip(gs.tolist(), gk.tolist()), key=lambda p: (-p[0], p[1]))[:k]
        assert list(zip(ts.tolist(), tk.tolist())) == exp


# ----------------------------------------------------------------- median ---

@pytest.mark.parametrize("seed", range(20))
def test_median_counting_definition(orc, seed):
    rng = np.random.default_rng(200 + seed)
    n = int(rng.integers(1, 65))
    rows = rand_rows32(rng, n, int(rng.integers(1, 6)), 10, extreme=(seed % 4 == 0))
    for i in range(0, n, 3):     # repeated values
        k, _, ts, p = rows[i]
        rows[i] = (k, 77, ts, p)
    t = rows32(rows)
    keys, rids = orc.extract(t, LAYOUT32)
    mk, mv = orc.median_by_key(keys, rids, t, LAYOUT32)
    assert mk.tolist() == sorted(set(r[0] for r in rows))
    for k, m in zip(mk.tolist(), mv.tolist()):
        vals = [r[1] for r in rows if r[0] == k]
        h = (len(vals) - 1) // 2
        assert sum(1 for v in vals if v < m) <= h < sum(1 for v in vals if v <= m)
        assert m == sorted(vals)[h]


# ------------------------------------------------------------------- join ---

@pytest.mark.parametrize("seed", range(25))
def test_join_nested_loops_and_closed_form(orc, seed):
    rng = np.random.default_rng(300 + seed)
    nl, nr = int(rng.integers(0, 65)), int(rng.integers(0, 65))
    nk = int(rng.integers(1, 12))
    L = rand_rows32(rng, nl, nk, 10, extreme=(seed % 5 == 0))
    R = rand_rows32(rng, nr, nk, 10)
    if seed % 2 and nl and nr:   # share keys across the two sides
        R = [(L[int(rng.integers(0, nl))][0], v, ts, p) for (k, v, ts, p) in R]
    tl, tr = rows32(L), rows32(R)
    lk, lr = orc.extract(tl, LAYOUT32)
    rk, rr = orc.extract(tr, LAYOUT32)
    cnt, sp, pairs, npairs = orc.join(lk, lr, rk, rr, tl, tr, LAYOUT32, 64 * 64)
    exp_pairs = []
    esp = 0
    for i, (k1, v1, _, _) in enumerate(L):
        for j, (k2, v2, _, _) in enumerate(R):
            if k1 == k2:
                exp_pairs.append((k1, i, j))
                esp = (esp + v1 * v2) % (1 << 64)
    exp_pairs.sort()
    assert cnt == len(exp_pairs) == npairs and sp == esp
    assert [tuple(p) for p in pairs.tolist()] == exp_pairs
    # closed forms: count = sum cL*cR, sumprod = sum SL*SR (mod 2^64)
    keysset = set(r[0] for r in L) & set(r[0] for r in R)
    cf = sum(sum(1 for r in L if r[0] == k) * sum(1 for r in R if r[0] == k) for k in keysset)
    sf = sum(sum(r[1] for r in L if r[0] == k) * sum(r[1] for r in R if r[0] == k)
             for k in keysset) % (1 << 64)
    assert cnt == cf and sp == sf


def test_join_capacity_reports_total(orc):
    t = rows32([(4, 1, 0, 0)] * 5)
    k, r = orc.extract(t, LAYOUT32)
    cnt, sp, pairs, npairs = orc.join(k, r, k, r, t, t, LAYOUT32, 3)
    assert cnt == 25 and npairs == 25 and len(pairs) == 3 and sp == 25


def test_join_no_match(orc):
    a = rows32([(1, 5, 0, 0), (2, 5, 0, 0)])
    b = rows32([(3, 5, 0, 0)])
    ak, ar = orc.extract(a, LAYOUT32)
    bk, br = orc.extract(b, LAYOUT32)
    cnt, sp, pairs, npairs = orc.join(ak, ar, bk, br, a, b, LAYOUT32, 4)
    assert (cnt, sp, npairs) == (0, 0, 0)


# ------------------------------------------------------------ materialize ---

def test_materialize_rows(orc):
    rng = np.random.default_rng(9)
    t = rows32(rand_rows32(rng, 50, 5, 10))
    rids = rng.permutation(50).astype(np.uint32)[:31]
    out = orc.materialize(rids, t, LAYOUT32).reshape(-1, 32)
    raw = t.numpy().view(np.uint8).reshape(-1, 32)
    for i, r in enumerate(rids):
        assert bytes(out[i]) == bytes(raw[r])


# -------------------------------------------------------------------- pwl ---

def test_pwl_fit_counts(orc):
    rng = np.random.default_rng(12)
    for n_seg in (1, 3, 16, 1024):
        for _ in range(5):
            n = int(rng.integers(1, 300))
            base = int(rng.integers(0, 1 << 62))
            keys = np.sort(np.uint64(base) + rng.integers(0, 1 << int(rng.integers(1, 62)),
                                                          size=n, dtype=np.uint64))
            kmin, kmax, knots = orc.pwl_fit(keys, n_seg)
            assert kmin == int(keys[0]) and kmax == int(keys[-1])
            span = kmax - kmin
            kl = [int(x) for x in keys.tolist()]
            for j in range(n_seg + 1):
                b = kmin + (span * j) // n_seg
                below = sum(1 for x in kl if x < b)
                assert knots[j] == np.float32(below / n)
            assert knots[0] == 0.0
            assert np.all(np.diff(knots) >= 0)


# ---------------------------------------------------------- window bundle ---

def test_window_aggregate_matches_primitives(orc):
    rows = datagen.gen_c2(1 << 14, seed=5, n_keys=300, span_ns=10 ** 4)
    g, tk, ts, cs = orc.window_aggregate(rows, LAYOUT32, 1000, 10, k=10, n_threads=3)
    keys, rids, off, oob = orc.partition(rows, LAYOUT32, 1000, 10)
    assert oob == 0
    for w in range(10):
        a, b = int(off[w]), int(off[w + 1])
        gk, gc, gs, gm = orc.reduce_by_key(keys[a:b], rids[a:b], rows, LAYOUT32)
        assert g[w] == len(gk)
        ek, es = orc.topk_by_sum(gk, gs, 10)
        assert np.array_equal(tk[w][:len(ek)], ek) and np.array_equal(ts[w][:len(es)], es)
