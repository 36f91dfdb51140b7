"""GPU tests of the serving loop: bundles admitted as slots and memory free
up, windows closed by watermarks (merge of the window's sorted runs, then the
query's operator), results compared window by window with the oracle, and
the same query's results alone and in a mix of concurrent queries (and with
rows kept on the host) are identical.  Back-pressure, late rows and early
watermark application are forced from the host."""
import numpy as np
import pytest
import torch

import datagen
from datagen.rows import LAYOUT32
from gpu_util import kpa_mod, need_gpu, say

pytestmark = pytest.mark.gpu

W = 10 ** 5          # window length (ns)
SPAN = 12 * W        # event-time span of a stream


@pytest.fixture(scope="module")
def K():
    need_gpu()
    return kpa_mod()


M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)


def fmix(z):
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
        return z ^ (z >> np.uint64(31))


def digest(key, a, b=None, c=None):
    z = np.zeros_like(key)
    b = z if b is None else b
    c = z if c is None else c
    with np.errstate(over="ignore"):
        return int(np.sum(fmix(key ^ fmix(a ^ fmix(b ^ fmix(c)))), dtype=np.uint64))


def u64col(rows, i):
    return rows[:, i].numpy().view(np.uint64)


def stream_rows(kind, n, seed, side=0):
    if kind == "sum":
        return datagen.gen_c2(n, seed=seed, n_keys=3000, span_ns=SPAN)
    return datagen.gen_c3(n, seed=seed, side=side, n_keys=20000, span_ns=SPAN)


def bundles(n, seed, lo=9, hi=13):
    rng = np.random.default_rng(seed)
    cuts = [0]
    while cuts[-1] < n:
        cuts.append(min(n, cuts[-1] + int(2 ** rng.uniform(lo, hi))))
    return list(zip(cuts[:-1], cuts[1:]))


def expected(orc, kind, rows, rows_r=None):
    """Per window (index -> summary) from the oracle's ordered-map operators."""
    out = {}
    ts = u64col(rows, 2)
    wins = set((ts // W).tolist())
    if rows_r is not None:
        wins |= set((u64col(rows_r, 2) // W).tolist())
    for w in sorted(wins):
        m = np.nonzero(ts // W == w)[0]
        keys = u64col(rows, 0)[m]
        rids = m.astype(np.uint32)
        if kind == "sum":
            gk, gc, gs, gm = orc.reduce_by_key(keys, rids, rows, LAYOUT32)
            tk, tsum = orc.topk_by_sum(gk, gs, 10)
            with np.errstate(over="ignore"):
                tot = int(np.sum(gs, dtype=np.uint64))
            out[w] = {"rows": (len(m), 0), "groups": len(gk), "total": tot,
                      "digest": digest(gk, gc, gs, gm), "top_key": list(map(int, tk)),
                      "top_sum": list(map(int, tsum))}
        elif kind == "median":
            gk, gmed = orc.median_by_key(keys, rids, rows, LAYOUT32)
            out[w] = {"rows": (len(m), 0), "groups": len(gk), "total": 0,
                      "digest": digest(gk, gmed), "top_key": [], "top_sum": []}
        else:
            tr = u64col(rows_r, 2)
            mr = np.nonzero(tr // W == w)[0]
            cnt, sp, _, _ = orc.join(keys, rids, u64col(rows_r, 0)[mr], mr.astype(np.uint32),
                                     rows, rows_r, LAYOUT32)
            out[w] = {"rows": (len(m), len(mr)), "groups": cnt, "total": sp, "digest": 0,
                      "top_key": [], "top_sum": []}
    return out


def summary(r):
    return {k: r[k] for k in ("rows", "groups", "total", "digest", "top_key", "top_sum")}


class Stream:
    """One query's input: rows in arrival order, cut into bundles."""

    def __init__(self, kind, n, seed):
        self.kind = kind
        self.rows = stream_rows(kind, n, seed)
        self.rows_r = stream_rows(kind, n + 101, seed + 1, side=1) if kind == "join" else None
        self.parts = [(0, a, b) for a, b in bundles(n, seed)]
        if self.rows_r is not None:
            self.parts += [(1, a, b) for a, b in bundles(n + 101, seed + 7)]
            self.parts.sort(key=lambda p: (p[1], p[0]))
        self.pinned = {}

    def side_rows(self, side):
        return self.rows if side == 0 else self.rows_r

    def bundle(self, i):
        side, a, b = self.parts[i]
        key = (side, a, b)
        if key not in self.pinned:
            self.pinned[key] = self.side_rows(side)[a:b].contiguous().pin_memory()
        return side, self.pinned[key]

    def rid_layout(self):
        return LAYOUT32

    def watermark_after(self, i):
        """Largest watermark that no later bundle violates: the smallest
        timestamp still to come."""
        rest = self.parts[i + 1:]
        if not rest:
            return SPAN + W
        return min(int(u64col(self.side_rows(s)[a:b], 2).min()) for s, a, b in rest)


def run(K, streams, order, **cfg):
    """Submits the streams' bundles in `order` (list of (stream index, bundle
    index)) with a watermark after every third bundle of a stream; returns
    {stream index: {window: summary}} and the server's stats."""
    srv = K.Server(budget_bytes=4 << 30, max_bundle_rows=1 << 14, **cfg)
    kinds = {"sum": K.KPA_Q_SUM, "median": K.KPA_Q_MEDIAN, "join": K.KPA_Q_JOIN}
    qids = [srv.add_query(kinds[s.kind], LAYOUT32, W, 0) for s in streams]
    for si, bi in order:
        s = streams[si]
        side, rows = s.bundle(bi)
        srv.submit(qids[si], rows, side=side)
        if bi % 3 == 2:
            srv.watermark(qids[si], s.watermark_after(bi))
    for si, s in enumerate(streams):
        srv.watermark(qids[si], SPAN + W)
    srv.drain(timeout_ms=60000)
    res = {si: {} for si in range(len(streams))}
    for r in srv.results():
        si = qids.index(r["query"])
        assert r["window"] not in res[si], "window closed twice"
        res[si][r["window"]] = summary(r)
    st = srv.stats()
    srv.close()
    return res, st


def order_alone(streams, si):
    return [(si, b) for b in range(len(streams[si].parts))]


def order_mixed(streams):
    out, pos = [], [0] * len(streams)
    while any(pos[i] < len(s.parts) for i, s in enumerate(streams)):
        for i, s in enumerate(streams):
            if pos[i] < len(s.parts):
                out.append((i, pos[i]))
                pos[i] += 1
    return out


@pytest.fixture(scope="module")
def streams():
    return [Stream("sum", 120000, 11), Stream("median", 90000, 21), Stream("join", 60000, 31)]


@pytest.fixture(scope="module")
def oracle_results(orc, streams):
    return [expected(orc, s.kind, s.rows, s.rows_r) for s in streams]


def check_against_oracle(res, exp):
    assert set(res) == set(exp), (sorted(res), sorted(exp))
    for w in exp:
        assert res[w] == exp[w], (w, res[w], exp[w])


@pytest.mark.parametrize("si", [0, 1, 2])
def test_alone_matches_oracle(K, streams, oracle_results, si):
    say(f"serve alone {streams[si].kind}")
    res, st = run(K, streams, order_alone(streams, si))
    check_against_oracle(res[si], oracle_results[si])
    assert st["late_rows"] == 0 and st["windows_closed"] == len(oracle_results[si])


@pytest.mark.parametrize("host_rows", [0, 1])
def test_mixed_equals_alone_and_oracle(K, streams, oracle_results, host_rows):
    say(f"serve mixed host_rows={host_rows}")
    res, st = run(K, streams, order_mixed(streams), rows_in_host=host_rows, slots=4)
    for si in range(len(streams)):
        check_against_oracle(res[si], oracle_results[si])
    assert st["p99_ms"] >= st["p50_ms"] > 0 and st["rows"] > 0


def test_backpressure_and_early_watermarks(K, streams, oracle_results):
    """A pool that holds only a few bundles beside the close reserve, one
    slot and a pending queue of two: admission must wait for closes, and
    watermarks queued behind a waiting bundle are applied early when safe; a
    non-blocking submit reports back-pressure."""
    s = streams[0]
    srv = K.Server(budget_bytes=80 << 20, max_bundle_rows=1 << 13, max_pending=2, slots=1,
                   reserve_pct=90)
    q = srv.add_query(K.KPA_Q_SUM, LAYOUT32, W, 0)
    refused = 0
    # cut the stream into bundles of at most 2^13 rows
    parts = bundles(s.rows.shape[0], 5, lo=11, hi=13)
    for i, (a, b) in enumerate(parts):
        rows = s.rows[a:b].contiguous().pin_memory()
        try:
            srv.submit(q, rows, blocking=False)
        except K.KpaError as e:
            assert e.code == K.KPA_EBUDGET
            refused += 1
            srv.submit(q, rows, blocking=True)
        nxt = parts[i + 1][0] if i + 1 < len(parts) else None
        wm = SPAN + W if nxt is None else int(u64col(s.rows[nxt:], 2).min())
        srv.watermark(q, wm)
    srv.drain(timeout_ms=60000)
    res = {r["window"]: summary(r) for r in srv.results()}
    st = srv.stats()
    srv.close()
    say(f"refused {refused}, waits {st['backpressure_waits']}")
    assert st["backpressure_waits"] > 0
    check_against_oracle(res, oracle_results[0])


def test_late_rows_are_counted_not_merged(K, streams):
    s = streams[0]
    ts = u64col(s.rows, 2)
    first = np.nonzero(ts < W)[0]          # rows of window 0
    srv = K.Server(budget_bytes=2 << 30, max_bundle_rows=1 << 17)
    q = srv.add_query(K.KPA_Q_SUM, LAYOUT32, W, 0)
    a = s.rows[first].contiguous().pin_memory()
    srv.submit(q, a)
    srv.watermark(q, W)                    # closes window 0
    srv.submit(q, a)                       # the same rows again: all late
    srv.watermark(q, 2 * W)
    srv.drain(timeout_ms=60000)
    res = srv.results()
    st = srv.stats()
    srv.close()
    assert len(res) == 1 and res[0]["window"] == 0 and res[0]["rows"][0] == len(first)
    assert st["late_rows"] == len(first)


def test_ingest_rebases_timestamps(K):
    rows = datagen.gen_c2(5000, seed=3, n_keys=100, span_ns=W).pin_memory()
    dev = torch.empty_like(rows, device="cuda")
    K.kpa_ingest_bundle(rows, LAYOUT32, dev, ts_add=7 * W + 3)
    torch.cuda.synchronize()
    got = dev.cpu()
    exp = rows.clone()
    exp[:, 2] += 7 * W + 3
    assert torch.equal(got, exp)


# ------------------------------------------------ per-key arrays, placement --

def run_collect(K, s, order, **cfg):
    srv = K.Server(max_bundle_rows=1 << 14, **cfg)
    kinds = {"sum": K.KPA_Q_SUM, "median": K.KPA_Q_MEDIAN, "join": K.KPA_Q_JOIN}
    q = srv.add_query(kinds[s.kind], LAYOUT32, W, 0)
    for bi in order:
        side, rows = s.bundle(bi)
        srv.submit(q, rows, side=side)
        if bi % 3 == 2:
            srv.watermark(q, s.watermark_after(bi))
    srv.watermark(q, SPAN + W)
    srv.drain(timeout_ms=60000)
    res = {r["window"]: r for r in srv.results()}
    st = srv.stats()
    tr = srv.trace()
    srv.close()
    return res, st, tr


@pytest.mark.parametrize("si", [0, 1])
def test_per_key_arrays_match_oracle(K, orc, streams, oracle_results, si):
    """keep_groups: each SUM / MEDIAN window result carries its per-key arrays,
    compared element by element with the oracle's ordered-map results."""
    s = streams[si]
    say(f"serve per-key arrays {s.kind}")
    res, st, _ = run_collect(K, s, range(len(s.parts)), budget_bytes=4 << 30, keep_groups=1)
    ts = u64col(s.rows, 2)
    assert set(res) == set(oracle_results[si])
    for w, r in res.items():
        m = np.nonzero(ts // W == w)[0]
        keys, rids = u64col(s.rows, 0)[m], m.astype(np.uint32)
        a = r["arrays"]
        if s.kind == "sum":
            ek, ec, es, em = orc.reduce_by_key(keys, rids, s.rows, LAYOUT32)
            assert np.array_equal(a["gkey"], ek) and np.array_equal(a["cnt"], ec)
            assert np.array_equal(a["sum"], es) and np.array_equal(a["max"], em)
        else:
            ek, emed = orc.median_by_key(keys, rids, s.rows, LAYOUT32)
            assert np.array_equal(a["gkey"], ek) and np.array_equal(a["median"], emed)


@pytest.mark.parametrize("si", [0, 2])
def test_host_placement_matches_oracle(K, streams, oracle_results, si):
    """Every bundle KPA in the pinned host pool (the capacity tier): the
    window closes read the runs over the host link; results are unchanged."""
    s = streams[si]
    say(f"serve host placement {s.kind}")
    res, st, _ = run_collect(K, s, range(len(s.parts)), budget_bytes=4 << 30,
                             host_pool_bytes=1 << 30, placement=K.KPA_PLACE_HOST)
    check_against_oracle({w: summary(r) for w, r in res.items()}, oracle_results[si])
    assert st["bundles_on_host"] == st["bundles"] > 0
    assert all(r["runs_host"] == r["runs"] for r in res.values())


def test_balanced_placement_under_capacity_pressure(K, orc):
    """Balanced placement when the open windows' KPAs exceed the device pool:
    8M rows (128 MB of sorted keys and values) against a device pool of about
    117 MB outside the close reserve, rows kept on the host, and the
    watermark held back until every bundle is in.  The pool fills, bundles
    spill to the host pool, the monitor moves the knob toward the host (k_low
    falls), and every window's result still equals the oracle's."""
    n = 8 << 20
    rows = stream_rows("sum", n, 61)
    exp = expected(orc, "sum", rows)
    parts = bundles(n, 61, lo=12, hi=14)
    say(f"serve balanced placement under pressure: {len(parts)} bundles")
    srv = K.Server(budget_bytes=160 << 20, max_bundle_rows=1 << 14, slots=2, rows_in_host=1,
                   host_pool_bytes=1 << 30, placement=K.KPA_PLACE_BALANCED, monitor_ms=1,
                   target_delay_ms=10000, max_pending=1 << 20)
    q = srv.add_query(K.KPA_Q_SUM, LAYOUT32, W, 0)
    pinned = [rows[a:b].contiguous().pin_memory() for a, b in parts]
    for r in pinned:
        srv.submit(q, r)
    srv.watermark(q, SPAN + W)             # every window closes only now
    srv.drain(timeout_ms=120000)
    res = {r["window"]: summary(r) for r in srv.results()}
    st = srv.stats()
    tr = srv.trace()
    srv.close()
    say(f"bundles {st['bundles']} on host {st['bundles_on_host']}, k_low {st['k_low']:.2f}, "
        f"samples {len(tr)}")
    check_against_oracle(res, exp)
    assert st["bundles_on_host"] > 0
    assert min(t["k_low"] for t in tr) < 1.0


def one_window_bundle(n, seed):
    """n rows whose timestamps all fall in window 0, pinned."""
    rows = stream_rows("sum", n, seed)
    rows[:, 2] = torch.arange(n, dtype=torch.int64) % (W // 2)
    return rows.contiguous().pin_memory()


def test_stalled_server_reports_instead_of_waiting(K):
    """Bundles of one window fill the pool outside the close reserve and no
    watermark comes: no close is queued, so only a watermark could free
    memory.  A blocking submit that finds the pending queue full returns
    KPA_EBUDGET instead of waiting for ever, so does drain, and the server
    still shuts down."""
    rows = one_window_bundle(1 << 13, 71)
    srv = K.Server(budget_bytes=80 << 20, max_bundle_rows=1 << 13, max_pending=2, slots=1,
                   reserve_pct=50)
    q = srv.add_query(K.KPA_Q_SUM, LAYOUT32, W, 0)
    say("serve stall: filling one window")
    err = None
    for i in range(2000):                  # the pool holds about 100 such bundles
        try:
            srv.submit(q, rows)
        except K.KpaError as e:
            err = e
            break
    assert err is not None and err.code == K.KPA_EBUDGET and "stalled" in str(err), err
    with pytest.raises(K.KpaError) as d:
        srv.drain(timeout_ms=20000)
    assert d.value.code == K.KPA_EBUDGET and "stalled" in str(d.value)
    st = srv.stats()
    srv.close()
    say(f"stalled after {i} bundles, {st['bundles']} admitted")
    assert 50 < st["bundles"] < 200


def test_close_short_of_memory_stops_the_server(K):
    """With no close reserve, a window whose bundles hold 60% of the pool
    cannot be merged (the close needs several times its runs' bytes).  The
    closer cannot wait for memory that only closes free: the server stops
    with KPA_EBUDGET and says which window, instead of hanging."""
    rows = one_window_bundle(1 << 13, 72)
    srv = K.Server(budget_bytes=80 << 20, max_bundle_rows=1 << 13, slots=1, reserve_pct=0,
                   rows_in_host=1, max_pending=4096)
    q = srv.add_query(K.KPA_Q_SUM, LAYOUT32, W, 0)
    say("serve close short of memory")
    for _ in range(360):                   # 360 x 2^13 rows x 16 B = 47 MB of runs
        srv.submit(q, rows)
    srv.watermark(q, W)
    with pytest.raises(K.KpaError) as d:
        srv.drain(timeout_ms=60000)
    srv.close()
    assert d.value.code == K.KPA_EBUDGET and "closing window 0" in str(d.value), d.value


def test_drain_time_limit_is_a_timeout(K):
    """drain with a time limit shorter than the work returns KPA_ETIMEOUT and
    the server runs on; a later drain finishes."""
    rows = one_window_bundle(1 << 16, 73)
    srv = K.Server(budget_bytes=1 << 30, max_bundle_rows=1 << 16, slots=1, max_pending=4096,
                   rows_in_host=1)
    q = srv.add_query(K.KPA_Q_SUM, LAYOUT32, W, 0)
    for _ in range(100):
        srv.submit(q, rows)
    srv.watermark(q, W)
    with pytest.raises(K.KpaError) as d:
        srv.drain(timeout_ms=1)
    assert d.value.code == K.KPA_ETIMEOUT
    srv.drain(timeout_ms=60000)
    res = srv.results()
    srv.close()
    assert len(res) == 1 and res[0]["rows"][0] == 100 << 16
