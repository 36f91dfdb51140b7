"""The serving workload at its full offered rate: Poisson-arriving bundles of
2^13..2^20 32-byte rows at 200M rows/s for 2 s over 16 queries (8 windowed
sums, 4 medians, 4 two-stream joins), 1 s windows with staggered origins, a
watermark every 100 ms of event time, a 64 GiB device budget, as the
benchmark's serving leg runs it.  One window of a sum, a median and a join
query, each wholly inside the run, is rebuilt on the host from the bundles
submitted to it and checked against the oracle (per-key arrays; join count
and sum of value products)."""
import numpy as np
import pytest
import torch

import datagen
from datagen.rows import LAYOUT32
from gpu_util import kpa_mod, need_gpu, say

pytestmark = pytest.mark.gpu

W = 10 ** 9


@pytest.fixture(scope="module")
def K():
    need_gpu()
    return kpa_mod()


def test_serving_full_rate_sampled_windows(K, orc):
    pool_rows = 1 << 25
    pools = []
    for kind, seed in (("sum", 52), ("c3", 53)):
        rows = (datagen.gen_c2(pool_rows, seed=seed, device="cuda") if kind == "sum"
                else datagen.gen_c3(pool_rows, seed=seed, device="cuda"))
        i = torch.arange(pool_rows, dtype=torch.int64, device="cuda")
        rows[:, 2] = datagen.uniform_int(datagen.splitmix64(54, 9, i), 10 ** 6)  # 1 ms jitter
        host = torch.empty(rows.shape, dtype=rows.dtype, pin_memory=True)
        host.copy_(rows)
        pools.append(host)
        del rows, i
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    srv = K.Server(budget_bytes=64 << 30, slots=8, rows_in_host=0, max_bundle_rows=1 << 20,
                   max_pending=1024, keep_groups=1)
    kinds = [K.KPA_Q_SUM] * 8 + [K.KPA_Q_MEDIAN] * 4 + [K.KPA_Q_JOIN] * 4
    qids = [srv.add_query(k, LAYOUT32, W, q * (W // 16)) for q, k in enumerate(kinds)]
    rate, duration = 200e6, 2.0
    rng = np.random.default_rng(55)
    lam = rate / ((2 ** 20 - 2 ** 13) / np.log(2 ** 7))
    subs = [[] for _ in qids]
    side_next = [0] * len(qids)
    last_wm = [0] * len(qids)
    t_next, n_sub = 0.0, 0
    import time
    start = time.perf_counter()
    while True:
        t_next += rng.exponential(1.0 / lam)
        if t_next > duration:
            break
        now = time.perf_counter() - start
        if t_next > now:
            time.sleep(t_next - now)
        nb = int(2 ** rng.uniform(13, 20))
        q = n_sub % len(qids)
        pi = 0 if kinds[q] == K.KPA_Q_SUM else 1
        o = int(rng.integers(0, pool_rows - nb))
        side = 0
        if kinds[q] == K.KPA_Q_JOIN:
            side = side_next[q]
            side_next[q] ^= 1
        ev = int(t_next * 1e9) + W
        srv.submit(qids[q], pools[pi][o:o + nb], side=side, ts_base=ev, ts_lo=0,
                   ts_hi=10 ** 6 - 1, blocking=True)
        subs[q].append((pi, o, nb, side, ev))
        n_sub += 1
        for qq in range(len(qids)):
            if ev - last_wm[qq] >= 10 ** 8:
                srv.watermark(qids[qq], ev)
                last_wm[qq] = ev
    end_ev = int(duration * 1e9) + 2 * W + 10 ** 6
    for qq in range(len(qids)):
        srv.watermark(qids[qq], end_ev)
    srv.drain(timeout_ms=120000)
    st = srv.stats()
    res = {}
    while True:
        r = srv.poll(0)
        if r is None:
            break
        res[(r["query"], r["window"])] = r
    srv.close()
    say(f"serving: {n_sub} bundles, {st['rows']} rows, {st['mrec_per_s']:.0f} Mrec/s, "
        f"{len(res)} windows, late rows {st['late_rows']}")
    assert st["late_rows"] == 0

    def window_rows(q, w, side):
        """The rows of query q's window w on one side, timestamps rebased."""
        lo, hi = q * (W // 16) + w * W, q * (W // 16) + (w + 1) * W
        parts = []
        for pi, o, nb, sd, ev in subs[q]:
            if sd != side or ev + 10 ** 6 <= lo or ev >= hi:
                continue
            r = pools[pi][o:o + nb].clone()
            r[:, 2] += ev
            ts = r[:, 2].numpy().view(np.uint64)
            m = (ts >= lo) & (ts < hi)
            parts.append(r[torch.from_numpy(m)])
        rows = torch.cat(parts) if parts else torch.empty((0, 4), dtype=torch.int64)
        return rows, rows[:, 0].numpy().view(np.uint64).copy(), np.arange(len(rows), dtype=np.uint32)

    # window 1 of each query below lies wholly inside the run's event times
    for q in (0, 8, 12):
        r = res[(qids[q], 1)]
        rows_l, kl, rl = window_rows(q, 1, 0)
        say(f"query {q} window 1: {len(kl)} rows (side 0)")
        assert int(r["rows"][0]) == len(kl)
        if kinds[q] == K.KPA_Q_SUM:
            sk, sr = orc.sort(kl, rl)
            ek, ec, es, em = orc.reduce_by_key(sk, sr, rows_l, LAYOUT32)
            a = r["arrays"]
            assert np.array_equal(a["gkey"], ek) and np.array_equal(a["cnt"], ec)
            assert np.array_equal(a["sum"], es) and np.array_equal(a["max"], em)
        elif kinds[q] == K.KPA_Q_MEDIAN:
            ek, emed = orc.median_by_key(kl, rl, rows_l, LAYOUT32)
            a = r["arrays"]
            assert np.array_equal(a["gkey"], ek) and np.array_equal(a["median"], emed)
        else:
            rows_r, kr, rr = window_rows(q, 1, 1)
            assert int(r["rows"][1]) == len(kr)
            c, s_, _, _ = orc.join(kl, rl, kr, rr, rows_l, rows_r, LAYOUT32)
            assert int(r["groups"]) == c and int(r["total"]) == s_
