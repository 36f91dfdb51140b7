"""Pins for the oracle's single-pass benchmarks and the remaining Table 2
primitives: brute force in plain Python on tiny inputs (written from the
definitions, not from the oracle), closed forms and invariants.  CPU only.

Each case plants the inputs where a plausible mistake shows: repeated values
(top-k is a multiset, unique count is not), sums past 2^64 (the window sum is
exact in 128 bits), keys equal to the average (the filter is strict), keys
missing from the update table, timestamps on window and slide edges."""
import struct
from fractions import Fraction

import numpy as np
import pytest

from datagen.rows import LAYOUT16, LAYOUT32

M64 = (1 << 64) - 1


def pack32(quads):
    return np.frombuffer(b"".join(struct.pack("<QQQQ", *q) for q in quads), dtype=np.uint8).copy()


def pack16(triples):
    return np.frombuffer(b"".join(struct.pack("<QII", *t) for t in triples),
                         dtype=np.uint8).copy()


def field(raw, rid, row_bytes, off, w):
    b = bytes(raw[rid * row_bytes + off:rid * row_bytes + off + w])
    return int.from_bytes(b, "little")


def random_quads(rng, n, n_keys, ts_span, val_hi=1 << 64, extreme=False):
    keys = [int(x) for x in rng.integers(0, 1 << 63, size=n_keys, dtype=np.uint64) * 2 + 1]
    if extreme:
        keys[0] = 0
        if n_keys > 1:
            keys[1] = M64
    out = []
    for i in range(n):
        k = keys[int(rng.integers(0, n_keys))]
        v = int(rng.integers(0, min(val_hi, 1 << 63)))
        if val_hi > (1 << 63) and rng.random() < 0.5:
            v |= 1 << 63
        if extreme and rng.random() < 0.2:
            v = M64 if val_hi > (1 << 63) else val_hi - 1
        out.append((k, v, int(rng.integers(0, ts_span)), i))
    return out


def kpa_of(quads, rids=None):
    rids = list(range(len(quads))) if rids is None else rids
    return (np.array([quads[r][0] for r in rids], dtype=np.uint64),
            np.array(rids, dtype=np.uint32))


# ------------------------------------------------------------ TopK per key --

@pytest.mark.parametrize("seed", range(30))
def test_topk_per_key_brute_force(orc, seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(0, 60))
    val_hi = [4, 1000, 1 << 64][seed % 3]           # 4: many repeated values
    q = random_quads(rng, n, int(rng.integers(1, 6)), 100, val_hi, extreme=seed % 5 == 0)
    perm = [int(x) for x in rng.permutation(n)]     # KPA order is free
    keys, rids = kpa_of(q, perm)
    k = int(rng.integers(1, 8))
    gk, gc, tn, tv = orc.topk_per_key(keys, rids, pack32(q), LAYOUT32, k)
    groups = {}
    for key, v, _, _ in q:
        groups.setdefault(key, []).append(v)
    assert gk.tolist() == sorted(groups)
    for g, key in enumerate(sorted(groups)):
        vals = sorted(groups[key], reverse=True)
        assert int(gc[g]) == len(vals)
        assert int(tn[g]) == min(k, len(vals))
        assert tv[g, :tn[g]].tolist() == vals[:k]
        assert all(int(x) == 0 for x in tv[g, tn[g]:])


def test_topk_per_key_keeps_repeats(orc):
    q = [(7, 5, 0, 0), (7, 9, 0, 0), (7, 9, 0, 0), (7, 1, 0, 0), (3, 2, 0, 0)]
    keys, rids = kpa_of(q)
    gk, gc, tn, tv = orc.topk_per_key(keys, rids, pack32(q), LAYOUT32, 3)
    assert gk.tolist() == [3, 7] and tn.tolist() == [1, 3]
    assert tv.tolist() == [[2, 0, 0], [9, 9, 5]]


# -------------------------------------------------------- unique per key ---

@pytest.mark.parametrize("seed", range(30))
def test_unique_count_brute_force(orc, seed):
    rng = np.random.default_rng(200 + seed)
    n = int(rng.integers(0, 70))
    q = random_quads(rng, n, int(rng.integers(1, 5)), 10, [3, 50, 1 << 64][seed % 3])
    keys, rids = kpa_of(q, [int(x) for x in rng.permutation(n)])
    gk, gu = orc.unique_count_by_key(keys, rids, pack32(q), LAYOUT32)
    groups = {}
    for key, v, _, _ in q:
        groups.setdefault(key, set()).add(v)
    assert gk.tolist() == sorted(groups)
    assert gu.tolist() == [len(groups[key]) for key in sorted(groups)]


def test_unique_count_u32_values(orc):
    t = [(5, 0xFFFFFFFF, 1), (5, 0xFFFFFFFF, 2), (5, 0, 3), (9, 1, 4)]
    raw = pack16(t)
    keys = np.array([x[0] for x in t], np.uint64)
    rids = np.arange(4, dtype=np.uint32)
    gk, gu = orc.unique_count_by_key(keys, rids, raw, LAYOUT16)
    assert gk.tolist() == [5, 9] and gu.tolist() == [2, 1]


# ------------------------------------------------- unkeyed window reduce ---

@pytest.mark.parametrize("seed", range(25))
def test_reduce_all_windows_brute_force(orc, seed):
    rng = np.random.default_rng(300 + seed)
    n = int(rng.integers(0, 80))
    W, nw, origin = int(rng.integers(1, 20)), int(rng.integers(1, 6)), int(rng.integers(0, 10))
    q = random_quads(rng, n, 3, origin + W * nw + 15, 1 << 64, extreme=True)
    c, lo, hi, mx, oob = orc.reduce_all_windows(pack32(q), LAYOUT32, W, nw, origin)
    ec, es, em, eoob = [0] * nw, [0] * nw, [0] * nw, 0
    for _, v, ts, _ in q:
        if ts < origin or (ts - origin) // W >= nw:
            eoob += 1
            continue
        w = (ts - origin) // W
        ec[w] += 1
        es[w] += v                      # Python ints: the exact sum
        em[w] = max(em[w], v)
    assert oob == eoob and c.tolist() == ec and mx.tolist() == em
    assert [int(a) + (int(b) << 64) for a, b in zip(lo, hi)] == es


def test_reduce_all_sum_carries_into_high_word(orc):
    q = [(1, M64, 0, 0), (1, M64, 1, 0), (1, 3, 2, 0)]
    c, lo, hi, mx, oob = orc.reduce_all_windows(pack32(q), LAYOUT32, 10, 1)
    total = 2 * M64 + 3
    assert (int(c[0]), int(lo[0]), int(hi[0])) == (3, total & M64, total >> 64)
    assert int(hi[0]) == 2 and int(mx[0]) == M64


# ------------------------------------------------------------------ select --

OPS = {">": lambda a, b: a > b, ">=": lambda a, b: a >= b, "<": lambda a, b: a < b,
       "<=": lambda a, b: a <= b, "==": lambda a, b: a == b, "!=": lambda a, b: a != b}


@pytest.mark.parametrize("seed", range(36))
def test_select_brute_force(orc, seed):
    rng = np.random.default_rng(400 + seed)
    op = list(OPS)[seed % 6]
    column = (seed // 6) % 2
    n = int(rng.integers(0, 50))
    q = random_quads(rng, n, 4, 10, 1 << 64, extreme=True)
    n_seg = int(rng.integers(1, 5))
    cuts = sorted(int(x) for x in rng.integers(0, n + 1, size=n_seg - 1))
    off = [0] + cuts + [n]
    keys, rids = kpa_of(q, [int(x) for x in rng.permutation(n)])
    num, den = [], []
    for s in range(n_seg):
        d = int(rng.integers(0, 4)) if seed % 3 else int(rng.integers(1, 1 << 63))
        den.append(d)
        # thresholds near x * den of a member so that '==' and the edges happen
        if off[s + 1] > off[s] and rng.random() < 0.7:
            i = int(rng.integers(off[s], off[s + 1]))
            x = int(keys[i]) if column == 0 else q[int(rids[i])][1]
            num.append(x * d + int(rng.integers(-1, 2)) if x * d > 0 else 0)
        else:
            num.append(int(rng.integers(0, 1 << 62)) << 64 | int(rng.integers(0, 1 << 62)))
    lo = np.array([v & M64 for v in num], np.uint64)
    hi = np.array([v >> 64 for v in num], np.uint64)
    ok, orr, oo = orc.select(keys, rids, np.array(off, np.uint64), lo, hi,
                             np.array(den, np.uint64), op, column, pack32(q), LAYOUT32)
    ek, er, eo = [], [], [0]
    for s in range(n_seg):
        for i in range(off[s], off[s + 1]):
            x = int(keys[i]) if column == 0 else q[int(rids[i])][1]
            if OPS[op](x * den[s], num[s]):
                ek.append(int(keys[i]))
                er.append(int(rids[i]))
        eo.append(len(ek))
    assert ok.tolist() == ek and orr.tolist() == er and oo.tolist() == eo


# --------------------------------------------------------- windowed filter --

@pytest.mark.parametrize("seed", range(25))
def test_window_filter_brute_force(orc, seed):
    rng = np.random.default_rng(500 + seed)
    W, nw = int(rng.integers(1, 10)), int(rng.integers(1, 5))
    na, nb = int(rng.integers(0, 40)), int(rng.integers(0, 40))
    qa = random_quads(rng, na, 5, W * nw + 3, 1 << 64, extreme=True)
    qb = random_quads(rng, nb, 6, W * nw + 3, 1 << 64, extreme=True)
    # plant B keys equal to an A window's exact average (must not pass)
    for i in range(0, nb, 5):
        w = qb[i][2] // W
        va = [v for _, v, ts, _ in qa if ts // W == w]
        if va and sum(va) % len(va) == 0:
            qb[i] = (sum(va) // len(va),) + qb[i][1:]
    rb = 1000
    ok, orr, oo = orc.window_filter(pack32(qa), pack32(qb), LAYOUT32, W, nw, 0, rb)
    avg = {}
    for w in range(nw):
        va = [v for _, v, ts, _ in qa if ts // W == w]
        avg[w] = Fraction(sum(va), len(va)) if va else None
    ek, er, eo = [], [], [0]
    for w in range(nw):
        for i, (key, _, ts, _) in enumerate(qb):
            if ts // W == w and avg[w] is not None and key > avg[w]:
                ek.append(key)
                er.append(rb + i)
        eo.append(len(ek))
    assert ok.tolist() == ek and orr.tolist() == er and oo.tolist() == eo


def test_window_filter_strict_at_average(orc):
    qa = [(0, 4, 0, 0), (0, 6, 1, 0)]                  # window 0 average 5
    qb = [(5, 0, 0, 0), (6, 0, 1, 0), (4, 0, 2, 0), (9, 0, 12, 0)]   # (9 in window 1: A empty)
    ok, orr, oo = orc.window_filter(pack32(qa), pack32(qb), LAYOUT32, 10, 2)
    assert ok.tolist() == [6] and orr.tolist() == [1] and oo.tolist() == [0, 1, 1]


# ------------------------------------------------------------- keyswap -----

@pytest.mark.parametrize("width", [4, 8])
def test_keyswap_reads_the_named_column(orc, width):
    rng = np.random.default_rng(600 + width)
    q = random_quads(rng, 33, 4, 1 << 40, 1 << 64)
    raw = pack32(q)
    rids = np.array([int(x) for x in rng.integers(0, 33, size=50)], np.uint32)
    for col_off in (8, 16, 20 if width == 4 else 24):
        got = orc.keyswap(rids, raw, 32, col_off, width)
        exp = [field(raw, int(r), 32, col_off, width) for r in rids]
        assert got.tolist() == exp


# -------------------------------------------- key update and write-back -----

@pytest.mark.parametrize("seed", range(15))
def test_key_update_brute_force(orc, seed):
    rng = np.random.default_rng(700 + seed)
    tk = [int(x) for x in rng.choice(1 << 20, size=int(rng.integers(0, 12)), replace=False)]
    tv = [int(x) for x in rng.integers(0, 1 << 63, size=len(tk))]
    keys = [int(rng.choice(tk)) if tk and rng.random() < 0.7 else int(rng.integers(0, 1 << 20))
            for _ in range(int(rng.integers(0, 40)))]
    table = dict(zip(tk, tv))
    got, miss = orc.key_update(np.array(keys, np.uint64), np.array(tk, np.uint64),
                               np.array(tv, np.uint64))
    assert got.tolist() == [table.get(k, k) for k in keys]
    assert miss == sum(1 for k in keys if k not in table)


def test_key_writeback_touches_only_its_column(orc):
    rng = np.random.default_rng(710)
    q = random_quads(rng, 20, 3, 100, 1 << 64)
    raw = pack32(q)
    rids = np.array([3, 0, 17, 9], np.uint32)
    keys = np.array([11, 22, M64, 0], np.uint64)
    out = orc.key_writeback(keys, rids, raw, 32, 24)
    exp = bytearray(raw.tobytes())
    for k, r in zip(keys.tolist(), rids.tolist()):
        exp[r * 32 + 24:r * 32 + 32] = int(k).to_bytes(8, "little")
    assert out.tobytes() == bytes(exp)


# -------------------------------------------- materialize + extract -------

def test_materialize_extract_definition(orc):
    rng = np.random.default_rng(800)
    q = random_quads(rng, 40, 5, 1 << 30, 1 << 64)
    raw = pack32(q)
    rids = np.array([int(x) for x in rng.integers(0, 40, size=25)], np.uint32)
    out, ok, orr = orc.materialize_extract(rids, raw, 32, 16, rid_base=7)
    exp_rows = b"".join(bytes(raw[int(r) * 32:int(r) * 32 + 32]) for r in rids)
    assert out.tobytes() == exp_rows
    assert ok.tolist() == [q[int(r)][2] for r in rids]       # column at 16 = timestamp
    assert orr.tolist() == list(range(7, 7 + 25))
    # the same bytes as Materialize alone, and Extract of its output
    assert np.array_equal(out, orc.materialize(rids, raw, LAYOUT32))


# ---------------------------------------------------------- sliding windows --

@pytest.mark.parametrize("seed", range(25))
def test_sliding_aggregate_brute_force(orc, seed):
    rng = np.random.default_rng(900 + seed)
    slide = int(rng.integers(1, 6))
    win = slide * int(rng.integers(1, 4)) + (int(rng.integers(0, slide)) if seed % 4 == 0 else 0)
    nw, origin = int(rng.integers(1, 6)), int(rng.integers(0, 5))
    n = int(rng.integers(0, 60))
    q = random_quads(rng, n, int(rng.integers(1, 5)), origin + slide * nw + win + 3, 1 << 64,
                     extreme=True)
    gk, gc, gs, gm, go = orc.sliding_aggregate(pack32(q), LAYOUT32, win, slide, nw, origin)
    ek, ec, es, em, eo = [], [], [], [], [0]
    for w in range(nw):
        lo = origin + w * slide
        agg = {}
        for key, v, ts, _ in q:
            if lo <= ts < lo + win:
                a = agg.setdefault(key, [0, 0, 0])
                a[0] += 1
                a[1] = (a[1] + v) & M64
                a[2] = max(a[2], v)
        for key in sorted(agg):
            ek.append(key); ec.append(agg[key][0]); es.append(agg[key][1]); em.append(agg[key][2])
        eo.append(len(ek))
    assert gk.tolist() == ek and gc.tolist() == ec and gs.tolist() == es and gm.tolist() == em
    assert go.tolist() == eo


def test_sliding_equals_tumbling_when_slide_is_length(orc):
    rng = np.random.default_rng(950)
    q = random_quads(rng, 200, 7, 50, 1 << 20)
    raw = pack32(q)
    gk, gc, gs, gm, go = orc.sliding_aggregate(raw, LAYOUT32, 10, 10, 5)
    keys, rids, off, oob = orc.partition(raw, LAYOUT32, 10, 5)
    for w in range(5):
        a, b = int(off[w]), int(off[w + 1])
        ek, ec, es, em = orc.reduce_by_key(keys[a:b], rids[a:b], raw, LAYOUT32)
        g0, g1 = int(go[w]), int(go[w + 1])
        assert gk[g0:g1].tolist() == ek.tolist() and gs[g0:g1].tolist() == es.tolist()
        assert gc[g0:g1].tolist() == ec.tolist() and gm[g0:g1].tolist() == em.tolist()


def test_thresholds_given_as_python_lists_stay_exact(orc):
    """Lists of Python ints at or above 2^63 reach the oracle exactly (numpy's
    default conversion of such a list is float64, which would round the
    threshold 2^63 + 1 down to 2^63 and let the key 2^63 pass)."""
    big = (1 << 63) + 1
    keys = np.array([big - 1, big, big + 1], np.uint64)
    rids = np.arange(3, dtype=np.uint32)
    ok, orr, oo = orc.select(keys, rids, [0, 3], [big], [0], [1], ">=")
    assert ok.tolist() == [big, big + 1] and orr.tolist() == [1, 2] and oo.tolist() == [0, 2]


# ------------------------------------------------------- full-row grouping --

@pytest.mark.parametrize("seed", range(20))
def test_sort_rows_windowed_brute_force(orc, seed):
    rng = np.random.default_rng(1000 + seed)
    W, nw, origin = int(rng.integers(1, 9)), int(rng.integers(1, 5)), int(rng.integers(0, 4))
    n = int(rng.integers(0, 50))
    q = random_quads(rng, n, int(rng.integers(1, 6)), origin + W * nw + 4, 1 << 64, extreme=True)
    raw = pack32(q)
    out, off, oob = orc.sort_rows_windowed(raw, LAYOUT32, W, nw, origin)

    def win(ts):
        return nw if ts < origin or (ts - origin) // W >= nw else (ts - origin) // W

    order = sorted(range(n), key=lambda i: (win(q[i][2]), q[i][0], i))   # stable: ties by row
    assert out.tobytes() == b"".join(bytes(raw[i * 32:(i + 1) * 32]) for i in order)
    counts = [sum(1 for i in range(n) if win(q[i][2]) == w) for w in range(nw + 1)]
    assert off.tolist() == [sum(counts[:w]) for w in range(nw + 1)]
    assert oob == counts[nw]


def test_sort_rows_then_scan_equals_kpa_grouping(orc):
    """Grouping on full rows reaches the KPA path's per-key results: the sorted
    rows of each window, scanned as a KPA with rids in row order, reduce to
    the same groups as partition + sort + reduce on (key, pointer) pairs."""
    rng = np.random.default_rng(1100)
    q = random_quads(rng, 300, 12, 40, 1 << 64, extreme=True)
    raw = pack32(q)
    out, off, oob = orc.sort_rows_windowed(raw, LAYOUT32, 10, 3)
    keys, rids, poff, poob = orc.partition(raw, LAYOUT32, 10, 3)
    assert oob == poob and off[:4].tolist() == poff.tolist()
    sk, sr = orc.sort_segmented(keys, rids, poff)
    for w in range(3):
        a, b = int(off[w]), int(off[w + 1])
        rk, rr = orc.extract(out[a * 32:b * 32], LAYOUT32)
        e1 = orc.reduce_by_key(rk, rr, out[a * 32:b * 32], LAYOUT32)
        e2 = orc.reduce_by_key(sk[a:b], sr[a:b], raw, LAYOUT32)
        assert all(np.array_equal(x, y) for x, y in zip(e1, e2))
