"""Benchmark of the KPA grouping hot path on one MI355X.

Default workload (windowed aggregation at scale): 2^28 rows of 32 bytes {u64
key Zipf s=1.1 over 2^20 distinct 64-bit keys, u64 value uniform [0, 2^20),
u64 timestamp ns over 10 s with +-1 ms disorder, u64 pad}, 10 tumbling 1 s
windows.  One step = partition the rows into window KPAs, sort every window's
KPA, count/sum/max per key, top-10 keys by sum per window, with the rows
already resident in device memory.  Prints one JSON line.

--workload c4: 4096 substreams with one window each, sizes log-uniform over
[2^10, 2^22) rows, rank-ordered Zipf keys whose exponent and offset drift from
epoch 0 (the models' training data) to epoch 1 (measured).  One step = extract
+ batched sort (learned or radix for the large windows) + count/sum/max per
key of every window, replayed as one captured graph.

  python bench.py [--steps K] [--warmup W] [--algo radix|learned] [--rows N]
                  [--workload c2|c4]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Mrec/s KPA group-by (learned vs radix sort), % HBM peak, p99 latency"
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per entry and launch of each pass: the bytes the pass must
# read and write for one entry, whatever the caches do.
PASS_BYTES = {
    "radix_pass": 24,      # read key+rid, write key+rid
    "radix_hist": 8,       # read key
    "part_pass": 44,       # read 32-byte row, write key+rid
    "part_hist": 32,       # read the row (its timestamp spans the row's cache line share)
    "reduce_main": 20,     # read key+rid, gather 8-byte value
    "reduce_summary": 8,   # read key (plus the last run's values)
}


COPY_GBS = None  # device copy rate on this GPU (read + write bytes per second), set in main


def measure_copy_rate(dev, mib=1024, reps=5):
    """Read+write GB/s of a plain device-to-device copy of `mib` MiB (torch
    copy_), event-timed: the practical ceiling of a pass that reads and
    writes the same bytes, reported beside the roofline's spec peak."""
    import torch
    src = torch.empty(mib << 20, dtype=torch.uint8, device=dev).fill_(1)
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return round(2 * (mib << 20) / (ms / 1000) / 1e9, 1)


RADIX_PASS_SOURCES = ("onesweep.hpp", "digit_sort.hpp", "radix.hip")
LEARNED_PASS_SOURCES = ("onesweep.hpp", "digit_sort.hpp", "learned.hip", "learned_internal.hpp")


def counted_traffic(kernel_row, summary="c2_radix_hbm_bytes.md", sources=RADIX_PASS_SOURCES):
    """HBM bytes per dispatch of a kernel from a committed counter summary
    (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when the scatter
    pass's sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, "paper_1901_01328_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if f"sha256 {h.hexdigest()[:16]}" not in text:
        return None
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) == 4 and cells[0] == kernel_row:
            return int((float(cells[2]) + float(cells[3])) * 1e6)
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--algo", choices=["radix", "learned"], default="radix")
    ap.add_argument("--rows", type=int, default=1 << 28)
    ap.add_argument("--cpu-rows", type=int, default=3 << 26,
                    help="rows of the oracle's CPU-baseline sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--workload", choices=["c2", "c3", "c4", "c5"], default="c2")
    ap.add_argument("--duration", type=float, default=30.0, help="c5: seconds of offered load")
    ap.add_argument("--rate", type=float, default=200e6, help="c5: offered records per second")
    ap.add_argument("--host-rows", action="store_true", help="c5: keep full rows in host memory")
    ap.add_argument("--c4-windows", type=int, default=4096)
    ap.add_argument("--c4-hi-log2", type=int, default=22)
    ap.add_argument("--no-tune", action="store_true", help="c4: default batch configuration")
    ap.add_argument("--probe-copy-mib", type=int, default=0,
                    help="first copy this many MiB device-to-device (calibrates HBM byte counters)")
    return ap.parse_args()


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {a.gpus} is not supported (windows and "
              "substreams would be sharded over GPUs, one huge window by key range; that is "
              "not built)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import datagen
    import paper_1901_01328_amd as P
    from datagen.rows import LAYOUT32
    K = P.load()
    from paper_1901_01328_amd.pipeline import WindowAggregation

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    global COPY_GBS
    if not a.probe_copy_mib:  # counter runs calibrate on their own first copy
        COPY_GBS = measure_copy_rate(dev)
    if a.probe_copy_mib:
        src = torch.empty(a.probe_copy_mib << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if a.workload == "c4":
        return bench_c4(a)
    if a.workload == "c5":
        return bench_c5(a)
    if a.workload == "c3":
        return bench_c3(a)
    n = a.rows
    n_win, W = 10, 10 ** 9
    t0 = time.time()
    rows = datagen.gen_c2(n, seed=2, device=dev)
    torch.cuda.synchronize()
    print(f"[bench] generated {n} rows on the GPU in {time.time() - t0:.1f} s", file=sys.stderr,
          flush=True)
    algo = K.KPA_SORT_LEARNED if a.algo == "learned" else K.KPA_SORT_RADIX
    pipe = WindowAggregation(n, LAYOUT32, W, n_win, algo=algo, k=10, device=dev)
    stream = torch.cuda.current_stream()
    for _ in range(a.warmup):
        pipe.step(rows)
    torch.cuda.synchronize()
    print(f"[bench] warmup done ({a.warmup} steps)", file=sys.stderr, flush=True)

    K.kpa_profile_enable(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(a.steps):
        pipe.step(rows)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    K.kpa_profile_collect()
    ms_step = ev0.elapsed_time(ev1) / a.steps
    ms_wall = wall * 1000 / a.steps
    value = n / (max(ms_step, ms_wall) / 1000.0) / 1e6
    print(f"[bench] timed {a.steps} steps: {ms_step:.3f} ms/step (events), {ms_wall:.3f} (wall)",
          file=sys.stderr, flush=True)

    passes = {}
    for name in K.kpa_profile_names():
        cnt, tot = K.kpa_profile_get(name)
        if cnt == 0:
            continue
        avg = tot / cnt
        entry = {"launches_per_step": cnt / a.steps, "avg_ms": round(avg, 4)}
        if name in PASS_BYTES:
            gbs = PASS_BYTES[name] * n / (avg / 1000.0) / 1e9
            entry["alg_GBps"] = round(gbs, 1)
            entry["hbm_frac"] = round(gbs / HBM_PEAK_GBS, 4)
        passes[name] = entry
    K.kpa_profile_enable(False)

    # Active radix passes: digits that vary inside a window are sorted; for
    # these 64-bit keys all eight do in every window.
    sk = pipe.skeys
    off = pipe.win_off.cpu().numpy().view(np.uint64)
    active = 0
    for p in range(8):
        for w in range(n_win):
            seg = sk[int(off[w]):int(off[w + 1])]
            if seg.numel() == 0:
                continue
            d = (seg >> (8 * p)) & 255
            if bool((d != d[0]).any()):
                active += 1
    dom = "radix_pass" if algo == K.KPA_SORT_RADIX else "learned_scatter"
    roof = None
    if dom in passes:
        launches = passes[dom]["launches_per_step"]
        avg_ms = passes[dom]["avg_ms"]
        bytes_per_launch = PASS_BYTES.get(dom, 24) * n * (active / n_win) / launches \
            if dom == "radix_pass" else PASS_BYTES.get(dom, 24) * n
        achieved = bytes_per_launch / (avg_ms / 1000.0) / 1e9
        traffic = None
        if n == 1 << 28:
            traffic = counted_traffic("k_ds_pass<RadixDF>") if dom == "radix_pass" else \
                counted_traffic("k_ds_pass<LearnedDF>", "c2_learned_hbm_bytes.md",
                                LEARNED_PASS_SOURCES)
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "copy_gbs": COPY_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": dom, "avg_ms": avg_ms, "bytes_per_launch": int(bytes_per_launch)}

    check = None
    cpu = None
    if not a.no_cpu or not a.no_check:
        import oracle
        m = min(a.cpu_rows, n)
        host = rows[:m].cpu()
        threads = min(n_win, os.cpu_count() or 1)
        t1 = time.perf_counter()
        g, tk, ts, cs = oracle.window_aggregate(host, LAYOUT32, W, n_win, k=10, n_threads=threads)
        dt = time.perf_counter() - t1
        cpu = {"value": round(m / dt / 1e6, 3), "unit": "Mrec/s", "cores": threads,
               "kind": "oracle", "sample": f"first {m} of {n} rows (all their windows), "
               f"ordered-map keyed aggregation + top-10, {dt:.1f} s"}
        # windows fully inside the sample must agree exactly with the GPU
        gs = pipe.gseg.cpu().numpy().view(np.uint64)
        tkg = pipe.top_key.cpu().numpy().view(np.uint64).reshape(n_win, 10)
        tsg = pipe.top_sum.cpu().numpy().view(np.uint64).reshape(n_win, 10)
        full = [w for w in range(n_win) if (w + 1) * n / n_win + n / 1000 < m]
        ok = all(int(gs[w + 1] - gs[w]) == int(g[w]) and np.array_equal(tkg[w], tk[w]) and
                 np.array_equal(tsg[w], ts[w]) for w in full)
        check = {"windows_checked": full, "groups_and_top10_match_oracle": bool(ok)}
        print(f"[bench] oracle sample: {dt:.1f} s on {threads} threads; check {check}",
              file=sys.stderr, flush=True)

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Mrec/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(max(ms_step, ms_wall), 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "windowed keyed aggregation: 2^28 32-byte rows, Zipf s=1.1 keys "
                   "over 2^20, 10 tumbling 1 s windows, count/sum/max per key + top-10 by sum",
                   "rows": n, "row_bytes": 32, "windows": n_win, "sort": a.algo},
        "roofline": roof,
        "cpu_baseline": cpu,
        "passes": passes,
        "check": check,
    }
    print(json.dumps(out), flush=True)


def kernel_passes(K, steps, n, pass_bytes):
    """Per-kernel launches per step, mean ms and algorithmic GB/s (recorded
    with events on each launch's own stream since the last profile enable)."""
    K.kpa_profile_collect()
    passes = {}
    for name in K.kpa_profile_names():
        cnt, tot = K.kpa_profile_get(name)
        if cnt == 0:
            continue
        avg = tot / cnt
        entry = {"launches_per_step": cnt / steps, "avg_ms": round(avg, 4)}
        if name in pass_bytes:
            gbs = pass_bytes[name] * n / (avg / 1000.0) / 1e9
            entry["alg_GBps"] = round(gbs, 1)
            entry["hbm_frac"] = round(gbs / HBM_PEAK_GBS, 4)
        passes[name] = entry
    return passes


def bench_c4(a):
    import concurrent.futures as cf

    import numpy as np
    import torch

    import datagen
    import oracle
    import paper_1901_01328_amd as P
    from datagen.rows import LAYOUT32
    from paper_1901_01328_amd.pipeline import BatchAggregation
    K = P.load()
    dev = torch.device("cuda:0")
    sizes = datagen.c4_window_sizes(a.c4_windows, hi_log2=a.c4_hi_log2)
    n = int(sizes.sum())
    n_seg = len(sizes)
    algo = K.KPA_SORT_LEARNED if a.algo == "learned" else K.KPA_SORT_RADIX
    t0 = time.time()
    rows = datagen.gen_c4(0, sizes, device=dev)
    torch.cuda.synchronize()
    print(f"[bench] c4 epoch 0: {n} rows in {n_seg} windows generated in {time.time() - t0:.1f} s",
          file=sys.stderr, flush=True)
    pipe = BatchAggregation(n, n_seg, LAYOUT32, device=dev,
                            learned_ws=algo == K.KPA_SORT_LEARNED)
    pipe.set_sizes(sizes)
    radix = K.batch_config(large_algo=K.KPA_SORT_RADIX)
    pipe.step(rows, cfg=radix)
    pipe.fit_models()                      # epoch 1's models: epoch 0's sorted windows
    datagen.gen_c4(1, sizes, out=rows)
    pipe.step(rows, cfg=radix)             # extracts epoch 1 (the tuner sorts pipe.keys)
    torch.cuda.synchronize()
    print(f"[bench] c4 epoch 1 generated; models fitted ({time.time() - t0:.1f} s)",
          file=sys.stderr, flush=True)
    if a.no_tune:
        cfg, tune_ms = K.batch_config(large_algo=algo), None
    else:
        cfg, tune_ms = K.kpa_batch_autotune(
            pipe.keys, pipe.rids, pipe.seg_off, large_algo=algo, n_cap=n,
            models=pipe.models if algo == K.KPA_SORT_LEARNED else None, reps=2,
            keys_out=pipe.skeys, rids_out=pipe.srids, ws=pipe.ws_sort)
        print(f"[bench] autotuned {cfg.as_dict()} ({tune_ms:.2f} ms sort)", file=sys.stderr,
              flush=True)
    stream = torch.cuda.Stream()
    graph = pipe.capture(rows, stream, cfg=cfg)
    for _ in range(a.warmup):
        graph.launch(stream)
    stream.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(a.steps):
        graph.launch(stream)
    ev1.record(stream)
    stream.synchronize()
    wall = time.perf_counter() - wall0
    ms_step = max(ev0.elapsed_time(ev1), wall * 1000) / a.steps
    value = n / (ms_step / 1000.0) / 1e6
    print(f"[bench] c4 timed {a.steps} graph replays: {ms_step:.3f} ms/step", file=sys.stderr,
          flush=True)
    # Per-kernel times: the same step run eagerly with event timing per launch.
    K.kpa_profile_enable(True)
    prof_steps = 2
    for _ in range(prof_steps):
        pipe.step(rows, stream=stream, cfg=cfg)
    stream.synchronize()
    c4_bytes = dict(PASS_BYTES, extract=44)
    passes = kernel_passes(K, prof_steps, n, c4_bytes)
    K.kpa_profile_enable(False)
    st = pipe.stats.cpu().numpy().tolist()
    graph.destroy()

    # Oracle: every 16th window (their rows copied to the host), per window
    # the ordered-map keyed aggregation; the GPU's groups of those windows
    # must match exactly.
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    sample = list(range(0, n_seg, 16))
    goff = pipe.gseg.cpu().numpy().view(np.uint64)
    gk, gc, gs, gm = (t.cpu().numpy().view(np.uint64) for t in
                      (pipe.gkey, pipe.g["cnt"], pipe.g["sum"], pipe.g["max"]))
    host = {j: rows[off[j]:off[j + 1]].cpu() for j in sample}
    threads = min(16, os.cpu_count() or 1)

    def one(j):
        r = host[j]
        keys, rids = oracle.extract(r, LAYOUT32)
        return j, oracle.reduce_by_key(keys, rids, r, LAYOUT32)

    t1 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(one, sample))
    dt = time.perf_counter() - t1
    m = int(sum(sizes[j] for j in sample))
    ok = True
    for j, (ek, ec, es, em) in res:
        a0, b0 = int(goff[j]), int(goff[j + 1])
        ok = ok and b0 - a0 == len(ek) and np.array_equal(gk[a0:b0], ek) and \
            np.array_equal(gc[a0:b0], ec) and np.array_equal(gs[a0:b0], es) and \
            np.array_equal(gm[a0:b0], em)
    check = {"windows_checked": len(sample), "groups_match_oracle": bool(ok)}
    cpu = {"value": round(m / dt / 1e6, 3), "unit": "Mrec/s", "cores": threads, "kind": "oracle",
           "sample": f"every 16th window ({len(sample)} windows, {m} rows): extract + "
           f"ordered-map count/sum/max per key, {dt:.1f} s"}
    dom = "radix_pass" if algo == K.KPA_SORT_RADIX else "learned_scatter"
    roof = None
    if dom in passes:
        # bytes: 24 per entry of the large windows that take part in a launch;
        # all of them for the learned scatter, the active windows for radix
        large = int(sizes[sizes > cfg.mid_cap].sum())
        pl = passes[dom]
        per_launch = 24 * large if dom == "learned_scatter" else None
        if per_launch is None:
            # C4 keys vary in bits 12..31 (plus carries of the offset): count
            # the radix passes each large window needs from its own keys
            sk = pipe.skeys
            act = 0
            for j in np.nonzero(sizes > cfg.mid_cap)[0]:
                seg = sk[int(off[j]):int(off[j + 1])]
                x = seg ^ seg[0]
                act += int(sizes[j]) * sum(1 for p in range(8)
                                           if bool((((x >> (8 * p)) & 255) != 0).any()))
            per_launch = 24 * act / pl["launches_per_step"]
        achieved = per_launch / (pl["avg_ms"] / 1000.0) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "copy_gbs": COPY_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": dom, "avg_ms": pl["avg_ms"], "bytes_per_launch": int(per_launch)}
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "Mrec/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"{n_seg} substream windows, log-uniform 2^10..2^{a.c4_hi_log2} "
                   "rows of 32 bytes, drifting rank-Zipf keys; extract + batched sort + "
                   "count/sum/max per key, one graph replay per step",
                   "rows": n, "windows": n_seg, "sort": a.algo, "batch_config": cfg.as_dict(),
                   "autotune_sort_ms": tune_ms},
        "roofline": roof, "cpu_baseline": cpu, "passes": passes, "sort_stats": st,
        "check": check,
    }
    print(json.dumps(out), flush=True)


def bench_c3(a):
    """Temporal join + median: two streams of 2^26 32-byte rows, keys uniform
    over 2^24 (one key table for both), values uniform over u64, 10 tumbling
    1 s windows.  One step = partition + sort both streams, lower median per
    key on both, merge-join per window (count, sum of products mod 2^64)."""
    import concurrent.futures as cf

    import numpy as np
    import torch

    import datagen
    import oracle
    import paper_1901_01328_amd as P
    from datagen.rows import LAYOUT32
    from paper_1901_01328_amd.pipeline import JoinMedian
    K = P.load()
    dev = torch.device("cuda:0")
    n = 1 << 26
    n_win, W = 10, 10 ** 9
    rows_l = datagen.gen_c3(n, seed=3, side=0, device=dev)
    rows_r = datagen.gen_c3(n, seed=3, side=1, device=dev)
    pipe = JoinMedian(n, n, LAYOUT32, W, n_win, device=dev)
    stream = torch.cuda.current_stream()
    for _ in range(a.warmup):
        pipe.step(rows_l, rows_r)
    torch.cuda.synchronize()
    K.kpa_profile_enable(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(a.steps):
        pipe.step(rows_l, rows_r)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_step = max(ev0.elapsed_time(ev1), wall * 1000) / a.steps
    passes = kernel_passes(K, a.steps, 2 * n, PASS_BYTES)
    K.kpa_profile_enable(False)
    value = 2 * n / (ms_step / 1000.0) / 1e6
    print(f"[bench] c3 timed {a.steps} steps: {ms_step:.3f} ms/step", file=sys.stderr, flush=True)
    # oracle: two windows (every entry of them), both operators
    L, R = pipe.side
    hl, hr = rows_l.cpu(), rows_r.cpu()
    cnt = pipe.join["count"].cpu().numpy().view(np.uint64)
    sp = pipe.join["sumprod"].cpu().numpy().view(np.uint64)
    checked, ok = [3, 7], True
    t1 = time.perf_counter()

    def win(rows, w):
        ts = rows[:, 2].numpy().view(np.uint64)
        m = np.nonzero(ts // W == w)[0]
        return rows[:, 0].numpy().view(np.uint64)[m], m.astype(np.uint32)

    def one(w):
        lk, lr = win(hl, w)
        rk, rr = win(hr, w)
        c, s_, _, _ = oracle.join(lk, lr, rk, rr, hl, hr, LAYOUT32)
        mk, mm = oracle.median_by_key(lk, lr, hl, LAYOUT32)
        return w, c, s_, mk, mm, len(lk) + len(rk)

    with cf.ThreadPoolExecutor(len(checked)) as ex:
        res = list(ex.map(one, checked))
    dt = time.perf_counter() - t1
    goff = L["med"]["gseg_off"].cpu().numpy().view(np.uint64)
    gk = L["med"]["gkey"].cpu().numpy().view(np.uint64)
    gm = L["med"]["gmed"].cpu().numpy().view(np.uint64)
    m_rows = 0
    for w, c, s_, mk, mm, nr in res:
        a0, b0 = int(goff[w]), int(goff[w + 1])
        ok = ok and int(cnt[w]) == c and int(sp[w]) == s_ and np.array_equal(gk[a0:b0], mk) \
            and np.array_equal(gm[a0:b0], mm)
        m_rows += nr
    check = {"windows_checked": checked, "join_and_left_median_match_oracle": bool(ok),
             "pairs_per_window": int(cnt[checked[0]])}
    cpu = {"value": round(m_rows / dt / 1e6, 3), "unit": "Mrec/s", "cores": len(checked),
           "kind": "oracle", "sample": f"windows {checked} of both streams ({m_rows} rows): "
           f"ordered-map join + median per key, {dt:.1f} s"}
    roof = None
    if "radix_pass" in passes:
        pl = passes["radix_pass"]
        per_launch = 24 * 2 * n * 8 / pl["launches_per_step"]   # all 8 digits vary
        achieved = per_launch / (pl["avg_ms"] / 1000.0) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "copy_gbs": COPY_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "radix_pass", "avg_ms": pl["avg_ms"], "bytes_per_launch": int(per_launch)}
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "Mrec/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "temporal join + median per key: 2 x 2^26 32-byte rows, keys "
                   "uniform over 2^24, 10 tumbling 1 s windows", "rows": 2 * n, "windows": n_win},
        "roofline": roof, "cpu_baseline": cpu, "passes": passes, "check": check,
    }
    print(json.dumps(out), flush=True)


def bench_c5(a):
    """Serving: Poisson-arriving bundles (sizes log-uniform 2^13..2^20 rows)
    at the offered rate over 16 queries (8 windowed sums, 4 medians, 4 joins
    whose bundles alternate sides), 1 s tumbling windows with origins
    staggered by 1/16 s, a watermark per query every 100 ms of event time.
    Bundles are replayed from pinned pools of pre-generated rows, moved to
    their event time at ingest.  Reports sustained Mrec/s and the p50/p99 of
    window-close-to-result latency."""
    import numpy as np
    import torch

    import datagen
    import paper_1901_01328_amd as P
    from datagen.rows import LAYOUT32
    K = P.load()
    dev = torch.device("cuda:0")
    pool_rows = 1 << 25
    t0 = time.time()
    pools = []
    for kind in ("sum", "c3"):
        rows = (datagen.gen_c2(pool_rows, seed=52, device=dev) if kind == "sum"
                else datagen.gen_c3(pool_rows, seed=53, device=dev))
        i = torch.arange(pool_rows, dtype=torch.int64, device=dev)
        rows[:, 2] = datagen.uniform_int(datagen.splitmix64(54, 9, i), 10 ** 6)  # 1 ms jitter
        host = torch.empty(rows.shape, dtype=rows.dtype, pin_memory=True)
        host.copy_(rows)
        pools.append(host)
        del rows, i
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    print(f"[bench] c5 pools of {pool_rows} rows generated in {time.time() - t0:.1f} s",
          file=sys.stderr, flush=True)
    W = 10 ** 9
    srv = K.Server(budget_bytes=64 << 30, slots=8, rows_in_host=1 if a.host_rows else 0,
                   max_bundle_rows=1 << 20, max_pending=1024)
    kinds = [K.KPA_Q_SUM] * 8 + [K.KPA_Q_MEDIAN] * 4 + [K.KPA_Q_JOIN] * 4
    qids = [srv.add_query(k, LAYOUT32, W, q * (W // 16)) for q, k in enumerate(kinds)]
    rng = np.random.default_rng(55)
    mean_rows = (2 ** 20 - 2 ** 13) / np.log(2 ** 7)      # log-uniform mean
    lam = a.rate / mean_rows                             # bundles per second
    side_next = [0] * len(qids)
    n_sub = 0
    last_wm = [0] * len(qids)
    start = time.perf_counter()
    t_next = 0.0
    last_print = 0.0
    while True:
        t_next += rng.exponential(1.0 / lam)
        if t_next > a.duration:
            break
        now = time.perf_counter() - start
        if t_next > now:
            time.sleep(t_next - now)
        n = int(2 ** rng.uniform(13, 20))
        q = n_sub % len(qids)
        pool = pools[0] if kinds[q] == K.KPA_Q_SUM else pools[1]
        off = int(rng.integers(0, pool_rows - n))
        side = 0
        if kinds[q] == K.KPA_Q_JOIN:
            side = side_next[q]
            side_next[q] ^= 1
        ev = int(t_next * 1e9) + W        # event time of the bundle (ns)
        srv.submit(qids[q], pool[off:off + n], side=side, ts_base=ev, ts_lo=0, ts_hi=10 ** 6 - 1)
        n_sub += 1
        # watermarks: every 100 ms of event time, at the latest arrival
        for qq in range(len(qids)):
            if ev - last_wm[qq] >= 10 ** 8:
                srv.watermark(qids[qq], ev)
                last_wm[qq] = ev
        if now - last_print > 5:
            st = srv.stats()
            print(f"[bench] c5 t={now:.1f}s bundles={n_sub} closed={st['windows_closed']} "
                  f"p99={st['p99_ms']:.1f} ms", file=sys.stderr, flush=True)
            last_print = now
    end_ev = int(a.duration * 1e9) + 2 * W + 10 ** 6
    for qq in range(len(qids)):
        srv.watermark(qids[qq], end_ev)
    srv.drain(timeout_ms=120000)
    st = srv.stats()
    res = srv.results()
    srv.close()
    lat = sorted(r["latency_ms"] for r in res)
    # the closes at the end (after the last watermark) are not steady state
    steady = [r["latency_ms"] for r in res if r["window"] < int(a.duration) - 1]
    steady.sort()
    pct = (lambda v, p: v[min(len(v) - 1, int(p * (len(v) - 1) + 0.5))] if v else None)
    out = {
        "metric": METRIC, "value": round(st["mrec_per_s"], 2), "unit": "Mrec/s", "n_gpus": 1,
        "steps": n_sub, "warmup": 0, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "serving: Poisson bundles of 2^13..2^20 32-byte rows at "
                   f"{a.rate / 1e6:.0f} M rec/s offered, 8 sum + 4 median + 4 join queries, "
                   "1 s windows, watermark every 100 ms", "duration_s": a.duration,
                   "rows_in_host": bool(a.host_rows), "budget_gib": 64},
        "latency_ms": {"p50": pct(steady, 0.5), "p99": pct(steady, 0.99), "max": lat[-1] if lat
                       else None, "windows": len(steady)},
        "server": st, "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
