"""GPU parity at the full sizes of the small, windowed and join workloads, in
the configurations the benchmark times, on sampled windows the oracle
computes in seconds (the many-substream workload's full-size test is in
test_gpu_c4.py):
  * 2^20 16-byte rows, one window: every group against the oracle;
  * 2^28 32-byte rows, 10 windows: windows 0 and 9 (groups and top-10) on
    the radix and learned routes, and the two routes' whole group output
    against each other;
  * 2 x 2^26 32-byte rows, 10 windows: join count, sum of products and both
    streams' medians for windows 0 and 9."""
import numpy as np
import pytest
import torch

import datagen
from datagen.rows import LAYOUT16, LAYOUT32
from gpu_util import kpa_mod, need_gpu, say, u64

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    need_gpu()
    return kpa_mod()


def _digest(*tensors, chunk=1 << 26):
    """Position-weighted wrapping sum of int64 words (odd weights: a single
    differing element always changes it)."""
    acc = torch.zeros((), dtype=torch.int64, device="cuda")
    for k, t in enumerate(tensors):
        t = t.reshape(-1).to(torch.int64)
        for s in range(0, t.numel(), chunk):
            x = t[s:s + chunk]
            i = torch.arange(s, s + x.numel(), dtype=torch.int64, device=x.device)
            acc += (x * (2 * i + 1 + 2 * k)).sum()
    return int(acc.item())


def _window_groups(pipe, w):
    gs = u64(pipe.gseg)
    g0, g1 = int(gs[w]), int(gs[w + 1])
    return [u64(t[g0:g1]) for t in (pipe.gkey, pipe.g["cnt"], pipe.g["sum"], pipe.g["max"])]


def test_c1_full_size(K, orc):
    from paper_1901_01328_amd.pipeline import WindowAggregation
    n = 1 << 20
    rows = datagen.gen_c1(n, seed=1)
    say(f"c1 full size: {n} 16-byte rows, one window")
    p = WindowAggregation(n, LAYOUT16, 10 ** 3, 1, k=10, device="cuda")
    p.step(rows.cuda())
    torch.cuda.synchronize()
    hk, hr, hoff, oob = orc.partition(rows, LAYOUT16, 10 ** 3, 1)
    assert oob == 0 and int(hoff[-1]) == n
    sk, sr = orc.sort(hk, hr)
    expect = orc.reduce_by_key(sk, sr, rows, LAYOUT16)
    assert len(expect[0]) == 1000
    for got, e in zip(_window_groups(p, 0), expect):
        assert np.array_equal(got, e)
    tk, ts = orc.topk_by_sum(expect[0], expect[2], 10)
    assert np.array_equal(u64(p.top_key)[:10], tk) and np.array_equal(u64(p.top_sum)[:10], ts)


def test_c2_full_size_sampled_windows(K, orc):
    from paper_1901_01328_amd.pipeline import WindowAggregation
    torch.cuda.empty_cache()
    n, W, nw = 1 << 28, 10 ** 9, 10
    rows = datagen.gen_c2(n, seed=2, device="cuda")
    say(f"c2 full size: {n} rows, {nw} windows")
    got, digests = {}, {}
    for algo in ("radix", "learned"):
        a = K.KPA_SORT_LEARNED if algo == "learned" else K.KPA_SORT_RADIX
        p = WindowAggregation(n, LAYOUT32, W, nw, algo=a, k=10, device="cuda")
        for _ in range(2 if algo == "learned" else 1):   # the learned route's models: step 1
            p.step(rows)
        torch.cuda.synchronize()
        say(f"c2 {algo} step done")
        G = int(p.gseg[-1].item())
        digests[algo] = _digest(p.gseg, *(t[:G] for t in (p.gkey, p.g["cnt"], p.g["sum"],
                                                         p.g["max"])))
        got[algo] = {w: (_window_groups(p, w), u64(p.top_key)[10 * w:10 * w + 10],
                         u64(p.top_sum)[10 * w:10 * w + 10]) for w in (0, nw - 1)}
        del p
        torch.cuda.empty_cache()
    assert digests["learned"] == digests["radix"]
    # the oracle on row ranges that hold the whole window (timestamps rise
    # with the row index, jittered by far less than n/1000 rows)
    for w in (0, nw - 1):
        lo = max(0, w * n // nw - n // 1000)
        hi = min(n, (w + 1) * n // nw + n // 1000)
        host = rows[lo:hi].cpu()
        hk, hr, hoff, _ = orc.partition(host, LAYOUT32, W, nw)
        a0, b0 = int(hoff[w]), int(hoff[w + 1])
        sk, sr = orc.sort(hk[a0:b0], hr[a0:b0])
        expect = orc.reduce_by_key(sk, sr, host, LAYOUT32)
        tk, ts = orc.topk_by_sum(expect[0], expect[2], 10)
        say(f"c2 window {w}: {b0 - a0} rows, {len(expect[0])} groups")
        for algo in ("radix", "learned"):
            groups, gtk, gts = got[algo][w]
            for x, e in zip(groups, expect):
                assert np.array_equal(x, e), (algo, w)
            assert np.array_equal(gtk, tk) and np.array_equal(gts, ts), (algo, w)
    del rows
    torch.cuda.empty_cache()


def test_c3_full_size_sampled_windows(K, orc):
    from paper_1901_01328_amd.pipeline import JoinMedian
    torch.cuda.empty_cache()
    n, W, nw = 1 << 26, 10 ** 9, 10
    rows_l = datagen.gen_c3(n, seed=3, side=0, device="cuda")
    rows_r = datagen.gen_c3(n, seed=3, side=1, device="cuda")
    say(f"c3 full size: 2 x {n} rows, {nw} windows")
    pipe = JoinMedian(n, n, LAYOUT32, W, nw, device="cuda")
    pipe.step(rows_l, rows_r)
    torch.cuda.synchronize()
    hl, hr = rows_l.cpu(), rows_r.cpu()
    cnt = u64(pipe.join["count"])
    sp = u64(pipe.join["sumprod"])

    def win(rows, w):
        ts = rows[:, 2].numpy().view(np.uint64)
        m = np.nonzero(ts // W == w)[0]
        return rows[:, 0].numpy().view(np.uint64)[m], m.astype(np.uint32)

    for w in (0, nw - 1):
        lk, lr = win(hl, w)
        rk, rr = win(hr, w)
        c, s_, _, _ = orc.join(lk, lr, rk, rr, hl, hr, LAYOUT32)
        say(f"c3 window {w}: {len(lk)} + {len(rk)} rows, {c} pairs")
        assert int(cnt[w]) == c and int(sp[w]) == s_, w
        for side, (k, r, rows) in zip(pipe.side, ((lk, lr, hl), (rk, rr, hr))):
            mk, mm = orc.median_by_key(k, r, rows, LAYOUT32)
            goff = u64(side["med"]["gseg_off"])
            a0, b0 = int(goff[w]), int(goff[w + 1])
            assert np.array_equal(u64(side["med"]["gkey"][a0:b0]), mk), w
            assert np.array_equal(u64(side["med"]["gmed"][a0:b0]), mm), w
    del pipe, rows_l, rows_r
    torch.cuda.empty_cache()
