"""Benchmark of the KPA grouping hot path on one MI355X.

Workload (windowed aggregation at scale): 2^28 rows of 32 bytes {u64 key Zipf
s=1.1 over 2^20 distinct 64-bit keys, u64 value uniform [0, 2^20), u64
timestamp ns over 10 s with +-1 ms disorder, u64 pad}, 10 tumbling 1 s
windows.  One step = partition the rows into window KPAs, sort every window's
KPA, count/sum/max per key, top-10 keys by sum per window, with the rows
already resident in device memory.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--algo radix|learned] [--rows N]
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
# Algorithmic bytes per entry and launch of each pass.
PASS_BYTES = {
    "radix_pass": 24,      # read key+rid, write key+rid
    "radix_hist": 8,       # read key
    "part_pass": 44,       # read 32-byte row, write key+rid
    "part_hist": 32,       # read the row (its timestamp spans the row's cache line share)
    "reduce_main": 20,     # read key+rid, gather 8-byte value
    "reduce_summary": 8,   # read key (plus the last run's values)
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--algo", choices=["radix", "learned"], default="radix")
    ap.add_argument("--rows", type=int, default=1 << 28)
    ap.add_argument("--cpu-rows", type=int, default=1 << 26,
                    help="rows of the oracle's CPU-baseline sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--probe-copy-mib", type=int, default=0,
                    help="first copy this many MiB device-to-device (calibrates HBM byte counters)")
    return ap.parse_args()


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {a.gpus} is not supported "
              "(the sharded design is described in DESIGN.md)", file=sys.stderr)
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
    if a.probe_copy_mib:
        src = torch.empty(a.probe_copy_mib << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
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
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
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


if __name__ == "__main__":
    main()
