"""Benchmark of the KPA grouping hot path on one MI355X.

Default workload (many substream windows with learned splitters): 4096
substreams with one window each, window sizes log-uniform over [2^10, 2^22)
rows (2,149,508,137 rows of 32 bytes {u64 key, u64 value uniform [0, 2^20),
u64 timestamp, u64 pad}), rank-ordered Zipf keys whose exponent (0.8 -> 1.4
over the substreams) and offset drift from epoch 0 to epoch 1.  Epoch 0 is
sorted and its sorted KPAs train one piecewise-linear CDF model per window;
epoch 1 is measured.  Two routes on the same epoch-1 bytes:
  learned: extract + batched sort (learned splitters for the large windows)
           + count/sum/max per key + the fit of next epoch's models;
  radix:   extract + batched sort (LSD radix) + count/sum/max per key.
Each step is one replay of a captured graph, with the rows resident in HBM.
`value` is the learned route's Mrec/s; the radix route is reported beside it.
Then the paper's two comparisons on this GPU (KPA vs grouping on full rows;
sort vs hash GroupBy; --no-ablations skips them) and a short serving leg
(Poisson bundles at 200M rec/s, p50/p99 window latency; --no-serve skips it).

Other workloads: --workload c2 (2^28 rows, 10 windows, one route), c3
(temporal join + median), c5 (serving alone).

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c4|c2|c3|c5]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Mrec/s KPA group-by (learned vs radix sort), % HBM peak, p99 latency"
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per entry of each pass: what the pass must read and
# write for one entry, whatever the caches do.  Passes over the large windows
# only (the batched sort's multi-workgroup class) are marked "large".
PASS_BYTES = {
    "radix_pass": 24,       # read key+rid, write key+rid (per entry of an active pass)
    "radix_hist": 8,        # read key
    "part_pass": 44,        # read 32-byte row, write key+rid
    "part_hist": 32,        # read the row (its timestamp spans the row's cache line share)
    "reduce_main": 20,      # read key+rid, gather 8-byte value
    "extract": 48,          # read 32-byte row, write key+value (the sort takes positions as rids)
    "learned_scatter": 24,  # read key+rid, write key+rid (entries of large windows)
    "learned_finish": 24,   # read key+rid, write key+rid (entries finished on chip)
    "learned_hist": 8,      # read key (entries of large windows)
}
# The same passes when the sort carries the staged value column beside the
# KPA (8 more bytes read and written per entry and pass) and the reduction
# reads keys and values in order.
PASS_BYTES_KV = dict(PASS_BYTES, radix_pass=40, learned_scatter=40, learned_finish=40,
                     reduce_main=16)
LARGE_ONLY = {"learned_scatter", "learned_finish", "learned_hist", "radix_hist"}
GROUP_BYTES = 32  # keyed reduction output per group: key, count, sum, max


COPY_GBS = None  # device copy rate on this GPU (read + write bytes per second), set in main


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


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


def counted_traffic(kernel_row, summary, sources):
    """HBM bytes per dispatch of a kernel from a committed counter summary
    (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when the kernel's
    sources changed since the counters were taken."""
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


# Counter summaries of the dominant kernels: (summary file, row, sources).
TRAFFIC = {
    ("c2", "radix_pass"): ("c2_radix_hbm_bytes.md", "k_ds_pass<RadixDF, false>",
                           ("onesweep.hpp", "digit_sort.hpp", "radix.hip")),
    ("c2", "learned_scatter"): ("c2_learned_hbm_bytes.md", "k_ds_pass<LearnedDF, false>",
                                ("onesweep.hpp", "digit_sort.hpp", "learned.hip",
                                 "learned_internal.hpp")),
    ("c4", "learned_scatter"): ("c4_learned_hbm_bytes.md", "k_ds_pass<LearnedDF, true>",
                                ("onesweep.hpp", "digit_sort.hpp", "learned.hip",
                                 "learned_internal.hpp")),
    ("c4", "reduce_main"): ("c4_reduce_hbm_bytes.md", "k_reduce_main_seq<false>",
                            ("reduce.hip", "reduce_internal.hpp")),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["c2", "c3", "c4", "c5", "ablations", "adapt", "ads",
                                           "models"],
                    default="c4")
    ap.add_argument("--algo", choices=["radix", "learned"], default="radix", help="c2 only")
    ap.add_argument("--rows", type=int, default=1 << 28, help="c2 rows")
    ap.add_argument("--cpu-rows", type=int, default=3 << 26,
                    help="c2: rows of the oracle's CPU-baseline sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="c4: skip the serving leg")
    ap.add_argument("--no-ablations", action="store_true",
                    help="c4: skip the KPA-vs-full-rows and sort-vs-hash legs")
    ap.add_argument("--serve-seconds", type=float, default=8.0, help="c4: serving leg length")
    ap.add_argument("--duration", type=float, default=30.0, help="c5: seconds of offered load")
    ap.add_argument("--rate", type=float, default=200e6, help="c5: offered records per second")
    ap.add_argument("--host-rows", action="store_true", help="c5: keep full rows in host memory")
    ap.add_argument("--c4-windows", type=int, default=4096)
    ap.add_argument("--c4-hi-log2", type=int, default=22)
    ap.add_argument("--c4-route", choices=["both", "learned", "radix"], default="both",
                    help="c4: routes to time (profiling runs of one route)")
    ap.add_argument("--no-tune", action="store_true", help="c4: default batch configuration")
    ap.add_argument("--no-graph", action="store_true",
                    help="c4: time eager steps instead of graph replays (counter runs)")
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
    import torch

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    global COPY_GBS
    if a.probe_copy_mib:  # counter runs calibrate on their own first copy
        src = torch.empty(a.probe_copy_mib << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    else:
        COPY_GBS = measure_copy_rate(dev)
    out = {"c4": bench_c4, "c2": bench_c2, "c3": bench_c3, "c5": bench_c5, "adapt": bench_adapt,
           "ads": bench_ads, "models": bench_models,
           "ablations": lambda a: {"metric": METRIC, "ablations": ablation_leg(a.steps, a.warmup)}
           }[a.workload](a)
    print(json.dumps(out), flush=True)
    if "error" in out:
        sys.exit(1)


def kernel_passes(K, steps, n, pass_bytes, n_large=None, extra=None, entries=None):
    """Per-kernel launches per step, mean ms and algorithmic GB/s (recorded
    with events on each launch's own stream since the last profile enable).
    extra: bytes per launch added to a kernel's per-entry bytes (the keyed
    reduction's group outputs).  entries: per-launch entry counts that
    replace n (the finishing pass works only on the entries of the chunks it
    sorts on chip: kpa_sort_stats.finished_on_chip)."""
    K.kpa_profile_collect()
    passes = {}
    for name in K.kpa_profile_names():
        cnt, tot = K.kpa_profile_get(name)
        if cnt == 0:
            continue
        avg = tot / cnt
        entry = {"launches_per_step": cnt / steps, "avg_ms": round(avg, 4)}
        if name in pass_bytes and name != "radix_pass":
            m = n_large if (name in LARGE_ONLY and n_large is not None) else n
            m = (entries or {}).get(name, m)
            gbs = (pass_bytes[name] * m + (extra or {}).get(name, 0)) / (avg / 1000.0) / 1e9
            entry["alg_GBps"] = round(gbs, 1)
            entry["hbm_frac"] = round(gbs / HBM_PEAK_GBS, 4)
        passes[name] = entry
    return passes


def roofline(passes, name, bytes_per_launch, traffic=None):
    pl = passes[name]
    achieved = bytes_per_launch / (pl["avg_ms"] / 1000.0) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "copy_gbs": COPY_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic, "kernel": name, "avg_ms": pl["avg_ms"],
            "launches_per_step": pl["launches_per_step"], "bytes_per_launch": int(bytes_per_launch)}


def dominant(passes):
    """The pass with the most time per step among those with a byte model."""
    best, t = None, -1.0
    for name, p in passes.items():
        if name in PASS_BYTES:
            tt = p["avg_ms"] * p["launches_per_step"]
            if tt > t:
                best, t = name, tt
    return best


def fingerprint(*tensors, chunk=1 << 27):
    """A position-dependent 64-bit digest of int tensors (wrapping sums of
    SplitMix64-finalized values): equal arrays give equal digests; a single
    differing element changes it except with probability about 2^-64."""
    import torch

    from datagen.rows import mix64
    acc = 0
    for k, t in enumerate(tensors):
        t = t.reshape(-1)
        for s in range(0, t.numel(), chunk):
            x = t[s:s + chunk].to(torch.int64)
            i = torch.arange(s, s + x.numel(), dtype=torch.int64, device=t.device)
            h = mix64(x ^ mix64(i * 2 + 1 + k * 0x51ED27)).sum()
            acc = (acc + int(h.item())) & ((1 << 64) - 1)
    return acc


def bench_c4(a):
    import numpy as np
    import torch

    import datagen
    import paper_1901_01328_amd as P
    from datagen.rows import LAYOUT32
    from paper_1901_01328_amd.pipeline import BatchAggregation
    K = P.load()
    dev = torch.device("cuda:0")
    sizes = datagen.c4_window_sizes(a.c4_windows, hi_log2=a.c4_hi_log2)
    n = int(sizes.sum())
    n_seg = len(sizes)
    t0 = time.time()
    rows = datagen.gen_c4(0, sizes, device=dev)
    torch.cuda.synchronize()
    log(f"c4 epoch 0: {n} rows in {n_seg} windows generated in {time.time() - t0:.1f} s")
    pipe = BatchAggregation(n, n_seg, LAYOUT32, device=dev, learned_ws=True)
    pipe.set_sizes(sizes)
    radix_cfg = K.batch_config(large_algo=K.KPA_SORT_RADIX)
    pipe.step(rows, cfg=radix_cfg)
    pipe.fit_models()                      # epoch 1's models: epoch 0's sorted windows
    datagen.gen_c4(1, sizes, out=rows)
    pipe.step(rows, cfg=radix_cfg)
    pipe.extract(rows)                     # epoch 1's keys: what the tuner sorts
    torch.cuda.synchronize()
    log(f"c4 epoch 1 generated; models fitted ({time.time() - t0:.1f} s)")

    routes = ["learned", "radix"] if a.c4_route == "both" else [a.c4_route]
    algo = {"learned": K.KPA_SORT_LEARNED, "radix": K.KPA_SORT_RADIX}
    cfgs, tune_ms = {}, {}
    for r in routes:
        if a.no_tune:
            cfgs[r], tune_ms[r] = K.batch_config(large_algo=algo[r]), None
        else:
            cfgs[r], tune_ms[r] = K.kpa_batch_autotune(
                pipe.keys, None, pipe.seg_off, large_algo=algo[r], n_cap=n,
                models=pipe.models if r == "learned" else None, reps=2,
                keys_out=pipe.skeys, rids_out=pipe.srids, ws=pipe.ws_sort)
            log(f"autotuned {r}: {cfgs[r].as_dict()} ({tune_ms[r]:.2f} ms sort)")

    stream = torch.cuda.Stream()
    res = {}
    for r in routes:
        fit = r == "learned"
        if a.no_graph:   # eager steps (counter collection does not follow graph replays)
            class _Eager:
                def launch(self, st):
                    pipe.step(rows, stream=st, cfg=cfgs[r], fit_next=fit)

                def destroy(self):
                    pass
            graph = _Eager()
        else:
            graph = pipe.capture(rows, stream, cfg=cfgs[r], fit_next=fit)
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
        ms = max(ev0.elapsed_time(ev1), wall * 1000) / a.steps
        graph.destroy()
        log(f"c4 {r}: {a.steps} {'eager steps' if a.no_graph else 'graph replays'}, "
            f"{ms:.3f} ms/step")
        res[r] = {"ms": ms, "value": n / (ms / 1000.0) / 1e6}

    # Per-kernel times: the same steps run eagerly with event timing per launch
    # on the launch's own stream (outside the timed region above).
    large = int(sizes[sizes > cfgs[routes[0]].mid_cap].sum())
    prof_steps = 2
    for r in routes:
        K.kpa_profile_enable(True)
        for _ in range(prof_steps):
            pipe.step(rows, stream=stream, cfg=cfgs[r], fit_next=(r == "learned"))
        stream.synchronize()
        # the learned route carries the value column through its sort, the
        # radix route's reduction follows the row ids (BatchAggregation's choice)
        table = PASS_BYTES_KV if r == "learned" else PASS_BYTES
        G = int(pipe.gseg[-1].item())
        res[r]["groups_total"] = G
        res[r]["sort_stats"] = pipe.stats.cpu().numpy().tolist()
        res[r]["passes"] = kernel_passes(K, prof_steps, n, table,
                                         n_large=int(sizes[sizes > cfgs[r].mid_cap].sum()),
                                         extra={"reduce_main": GROUP_BYTES * G},
                                         entries={"learned_finish": res[r]["sort_stats"][1]})
        K.kpa_profile_enable(False)
        # outputs of this route: whole-array digests, and the sampled windows' groups
        stream.synchronize()
        G = int(pipe.gseg[-1].item())
        res[r]["digest"] = {"sorted_kpa": fingerprint(pipe.skeys, pipe.srids),
                            "groups": fingerprint(pipe.gseg, *(t[:G] for t in (
                                pipe.gkey, pipe.g["cnt"], pipe.g["sum"], pipe.g["max"])))}
        off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        goff = pipe.gseg.cpu().numpy().view(np.uint64)
        sample = list(range(0, n_seg, 16))
        grp = {}
        for j in sample:
            g0, g1 = int(goff[j]), int(goff[j + 1])
            grp[j] = tuple(t[g0:g1].cpu().numpy().view(np.uint64).copy() for t in
                           (pipe.gkey, pipe.g["cnt"], pipe.g["sum"], pipe.g["max"]))
        res[r]["groups"] = grp

    # Active radix passes of the large windows (their keys' varying bytes)
    sk = pipe.skeys
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    act = 0
    for j in np.nonzero(sizes > cfgs[routes[-1]].mid_cap)[0]:
        seg = sk[int(off[j]):int(off[j + 1])]
        x = seg ^ seg[0]
        act += int(sizes[j]) * sum(1 for p in range(8) if bool((((x >> (8 * p)) & 255) != 0).any()))

    # Oracle: every 16th window, per-key count/sum/max, compared with both routes
    check, cpu = None, None
    sample = list(range(0, n_seg, 16))
    if not (a.no_check and a.no_cpu):
        import oracle
        host = {j: rows[off[j]:off[j + 1]].cpu() for j in sample}
        threads = min(16, os.cpu_count() or 1)

        def one(j):
            rr = host[j]
            keys, rids = oracle.extract(rr, LAYOUT32)
            return j, oracle.reduce_by_key(keys, rids, rr, LAYOUT32)

        t1 = time.perf_counter()
        with cf.ThreadPoolExecutor(threads) as ex:
            ores = dict(ex.map(one, sample))
        dt = time.perf_counter() - t1
        m = int(sum(sizes[j] for j in sample))
        check = {"windows_checked": len(sample), "rows_checked": m}
        for r in routes:
            ok = all(len(ores[j][0]) == len(res[r]["groups"][j][0]) and
                     all(np.array_equal(x, y) for x, y in zip(res[r]["groups"][j], ores[j]))
                     for j in sample)
            check[f"{r}_per_key_arrays_match_oracle"] = bool(ok)
        if len(routes) == 2:
            check["learned_equals_radix"] = {
                k: res["learned"]["digest"][k] == res["radix"]["digest"][k]
                for k in ("sorted_kpa", "groups")}
        cpu = {"value": round(m / dt / 1e6, 3), "unit": "Mrec/s", "cores": threads,
               "host_cores": os.cpu_count(), "kind": "oracle",
               "sample": f"every 16th window ({len(sample)} windows, {m} rows): extract + "
               f"ordered-map count/sum/max per key, {dt:.1f} s on {threads} threads"}
        log(f"oracle: {dt:.1f} s on {threads} threads; check {check}")

    # Roofline of the dominant kernel of the headline route
    head = routes[0]
    passes = res[head]["passes"]
    dom = dominant(passes)
    roof = None
    if dom:
        pl = passes[dom]
        tb = PASS_BYTES_KV if head == "learned" else PASS_BYTES
        if dom == "radix_pass":
            per_launch = tb[dom] * act / pl["launches_per_step"]
        elif dom in LARGE_ONLY:
            per_launch = tb[dom] * large
        else:
            per_launch = tb[dom] * n + (GROUP_BYTES * res[head]["groups_total"]
                                        if dom == "reduce_main" else 0)
        tr = TRAFFIC.get(("c4", dom))
        traffic = counted_traffic(tr[1], tr[0], tr[2]) if tr else None
        roof = roofline(passes, dom, per_launch, traffic)

    serving, ablations = None, None
    del pipe, rows, sk
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    if not a.no_ablations:
        ablations = ablation_leg()
    if not a.no_serve:
        serving = serve_leg(a.rate, a.serve_seconds, host_rows=False)

    out = {
        "metric": METRIC, "value": round(res[head]["value"], 2), "unit": "Mrec/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(res[head]["ms"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"{n_seg} substream windows (sizes log-uniform over "
                   f"[2^10, 2^{a.c4_hi_log2}), {n} rows of 32 bytes), drifting rank-Zipf "
                   "keys, PWL models fitted on the previous epoch; extract + batched sort carrying "
                   "the value column + count/sum/max per key (+ next models' fit on the learned route), one "
                   "graph replay per step", "route": head, "rows": n, "windows": n_seg,
                   "batch_config": cfgs[head].as_dict(), "autotune_sort_ms": tune_ms[head]},
        "roofline": roof, "cpu_baseline": cpu, "check": check,
        "passes": passes, "sort_stats": res[head]["sort_stats"],
    }
    if len(routes) == 2:
        rr = res["radix"]
        out["radix"] = {"value": round(rr["value"], 2), "unit": "Mrec/s",
                        "ms_per_step": round(rr["ms"], 4), "batch_config": cfgs["radix"].as_dict(),
                        "passes": rr["passes"]}
        out["speedup_learned_vs_radix"] = round(rr["ms"] / res["learned"]["ms"], 4)
        rd = dominant(rr["passes"])
        if rd == "radix_pass":
            out["radix"]["roofline"] = roofline(
                rr["passes"], rd, PASS_BYTES[rd] * act / rr["passes"][rd]["launches_per_step"])
        elif rd:
            m = int(sizes[sizes > cfgs["radix"].mid_cap].sum()) if rd in LARGE_ONLY else n
            out["radix"]["roofline"] = roofline(
                rr["passes"], rd, PASS_BYTES[rd] * m + (GROUP_BYTES * rr["groups_total"]
                                                       if rd == "reduce_main" else 0))
    if serving is not None:
        out["serving"] = serving
    if ablations is not None:
        out["ablations"] = ablations
    return out


def timed(fn, steps, warmup):
    """Mean ms of fn() over `steps` calls after `warmup`, event- and wall-timed
    on the current stream (the larger of the two)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return max(e0.elapsed_time(e1), (time.perf_counter() - w0) * 1000) / steps


def ablation_leg(steps=5, warmup=2):
    """The paper's two comparisons on this GPU, each against the KPA path on the
    same bytes, with identical outputs:
    * KPA vs full-row grouping (the design without KPAs, Sec. 7.3): 2^28
      32-byte rows of the windowed workload, count/sum/max per key and top-10
      per window, either by partition + KPA sort + keyed reduction or by
      ordering the rows themselves by (window, key) and scanning them;
    * sort vs hash GroupBy (Sec. 2.2): 10^8 16-byte rows {u64 key, u64 value},
      count/sum/max per key, by extract + KPA sort + keyed reduction or by an
      open-addressing hash table; with about 100 values per key (the paper's
      setting: the table fits the 256 MB last-level cache) and with about 1.5
      values per key (the table does not)."""
    import numpy as np
    import torch

    import datagen
    import paper_1901_01328_amd as P
    from datagen.rows import LAYOUT32, RowLayout
    from paper_1901_01328_amd.pipeline import VALUE_COLUMN, WindowAggregation
    K = P.load()
    dev = torch.device("cuda:0")
    out = {}
    # ---- KPA vs full rows
    n, n_win, W = 1 << 28, 10, 10 ** 9
    rows = datagen.gen_c2(n, seed=2, device=dev)
    kpa = WindowAggregation(n, LAYOUT32, W, n_win, k=10, device=dev)
    ms_kpa = timed(lambda: kpa.step(rows), steps, warmup)
    i64 = dict(dtype=torch.int64, device=dev)
    srows = torch.empty(n * 4, **i64)
    off = torch.empty(n_win + 1, **i64)
    oob = torch.empty(1, **i64)
    nb = K._ws_size("kpa_reduce_by_key_workspace_size", n, n_win)
    ws_red = torch.empty(nb, dtype=torch.uint8, device=dev)
    c = __import__("ctypes").c_size_t(0)
    K._call("kpa_sort_rows_windowed_workspace_size", n, 32, __import__("ctypes").byref(c))
    ws_rows = torch.empty(int(c.value), dtype=torch.uint8, device=dev)
    keys = torch.empty(n, **i64)
    rids = torch.empty(n, dtype=torch.int32, device=dev)
    gk = torch.empty(n, **i64)
    g = {w: torch.empty(n, **i64) for w in ("cnt", "sum", "max")}
    gseg = torch.empty(n_win + 1, **i64)
    tk = torch.empty(n_win * 10, **i64)
    tsum = torch.empty(n_win * 10, **i64)
    tn = torch.empty(n_win, dtype=torch.int32, device=dev)
    ws_top = torch.empty(K._ws_size("kpa_topk_by_sum_workspace_size", n, n_win),
                         dtype=torch.uint8, device=dev)

    def full_rows():
        K.kpa_sort_rows_windowed(rows, LAYOUT32, W, n_win, n=n, out_rows=srows, out_win_off=off,
                                 out_oob=oob, ws=ws_rows)
        K.kpa_extract(srows, LAYOUT32, out_keys=keys, out_rids=rids, n=n)
        K.kpa_reduce_by_key(keys, rids, off, srows, LAYOUT32, n_cap=n, ws=ws_red,
                            outs=dict(g, gkey=gk, gseg_off=gseg))
        K.kpa_topk_by_sum(gk, g["sum"], gseg, k=10, g_cap=n, ws=ws_top,
                          outs={"key": tk, "sum": tsum, "n": tn})

    ms_rows = timed(full_rows, steps, warmup)
    G = int(gseg[-1].item())
    same = (torch.equal(gseg, kpa.gseg) and torch.equal(gk[:G], kpa.gkey[:G]) and
            all(torch.equal(g[w][:G], kpa.g[w][:G]) for w in g) and
            torch.equal(tk, kpa.top_key) and torch.equal(tsum, kpa.top_sum))
    out["kpa_vs_full_rows"] = {
        "workload": "2^28 32-byte rows, Zipf keys over 2^20, 10 windows, count/sum/max per key "
                    "+ top-10 by sum", "kpa_ms": round(ms_kpa, 3), "full_rows_ms": round(ms_rows, 3),
        "kpa_mrec_per_s": round(n / ms_kpa / 1e3, 1),
        "full_rows_mrec_per_s": round(n / ms_rows / 1e3, 1),
        "kpa_speedup": round(ms_rows / ms_kpa, 3), "outputs_identical": bool(same)}
    log(f"ablation KPA vs full rows: {out['kpa_vs_full_rows']}")
    del rows, kpa, srows, keys, rids, gk, g, ws_rows, ws_red
    torch.cuda.empty_cache()
    # ---- sort vs hash GroupBy
    KV16 = RowLayout(16, 0, 8, 8, 8, 8)
    n = 10 ** 8
    res = []
    for n_keys in (1 << 20, 1 << 26):
        i = torch.arange(n, dtype=torch.int64, device=dev)
        table = datagen.key_table(n_keys, 77, dev)
        kv = torch.empty((n, 2), **i64)
        kv[:, 0] = table[datagen.uniform_int(datagen.splitmix64(78, 1, i), n_keys)]
        kv[:, 1] = datagen.splitmix64(78, 2, i)
        del i, table
        keys = torch.empty(n, **i64)
        rids = torch.empty(n, dtype=torch.int32, device=dev)
        vals = torch.empty(n, **i64)
        sk = torch.empty(n, **i64)
        sr = torch.empty(n, dtype=torch.int32, device=dev)
        soff = torch.tensor([0, n], **i64)
        ws_sort = torch.empty(K.kpa_sort_workspace_size(n, 1), dtype=torch.uint8, device=dev)
        ws_red = torch.empty(K._ws_size("kpa_reduce_by_key_workspace_size", n, 1),
                             dtype=torch.uint8, device=dev)
        gk = torch.empty(n, **i64)
        g = {w: torch.empty(n, **i64) for w in ("cnt", "sum", "max")}
        gseg = torch.empty(2, **i64)

        def by_sort():
            K.kpa_extract(kv, KV16, out_keys=keys, out_rids=rids, out_vals=vals, n=n)
            K.kpa_sort_segmented(keys, rids, soff, n_cap=n, keys_out=sk, rids_out=sr, ws=ws_sort)
            K.kpa_reduce_by_key(sk, sr, soff, vals, VALUE_COLUMN, n_cap=n, ws=ws_red,
                                outs=dict(g, gkey=gk, gseg_off=gseg))

        cap = 1 << int(np.ceil(np.log2(2 * n_keys)))
        ws_hash = torch.empty(K._ws_size("kpa_hash_groupby_workspace_size", cap),
                              dtype=torch.uint8, device=dev)
        ho = {name: torch.empty(n_keys + 1, **i64) for name in ("gkey", "cnt", "sum", "max")}
        ho["ngroups"] = torch.empty(1, **i64)

        def by_hash():
            K.kpa_hash_groupby(kv, KV16, cap, g_cap=n_keys + 1, n=n, outs=ho, ws=ws_hash)

        ms_sort = timed(by_sort, steps, warmup)
        ms_hash = timed(by_hash, steps, warmup)
        G = int(gseg[-1].item())
        Gh = int(ho["ngroups"].item())
        same = G == Gh
        if same:
            hk, order = torch.sort(ho["gkey"][:Gh].view(torch.int64) ^ (-(1 << 63)))
            same = torch.equal(gk[:G], ho["gkey"][:Gh][order]) and all(
                torch.equal(g[w][:G], ho[w][:Gh][order]) for w in g)
        res.append({"rows": n, "distinct_keys": G, "values_per_key": round(n / max(G, 1), 1),
                    "hash_table_mib": round(cap * 32 / 2 ** 20, 1), "sort_ms": round(ms_sort, 3),
                    "hash_ms": round(ms_hash, 3), "sort_speedup": round(ms_hash / ms_sort, 3),
                    "outputs_identical": bool(same)})
        log(f"ablation sort vs hash: {res[-1]}")
        del kv, keys, rids, vals, sk, sr, ws_sort, ws_red, gk, g, ws_hash, ho
        torch.cuda.empty_cache()
    out["sort_vs_hash"] = {"workload": "10^8 16-byte rows {u64 key, u64 value}, count/sum/max "
                           "per key; sort = extract + KPA radix sort + keyed reduction (groups in "
                           "key order), hash = open-addressing table (groups in table order)",
                           "points": res}
    return out


def bench_c2(a):
    import numpy as np
    import torch

    import datagen
    import paper_1901_01328_amd as P
    from datagen.rows import LAYOUT32
    from paper_1901_01328_amd.pipeline import WindowAggregation
    K = P.load()
    dev = torch.device("cuda:0")
    n = a.rows
    n_win, W = 10, 10 ** 9
    t0 = time.time()
    rows = datagen.gen_c2(n, seed=2, device=dev)
    torch.cuda.synchronize()
    log(f"generated {n} rows on the GPU in {time.time() - t0:.1f} s")
    algo = K.KPA_SORT_LEARNED if a.algo == "learned" else K.KPA_SORT_RADIX
    pipe = WindowAggregation(n, LAYOUT32, W, n_win, algo=algo, k=10, device=dev)
    stream = torch.cuda.current_stream()
    for _ in range(a.warmup):
        pipe.step(rows)
    torch.cuda.synchronize()
    # timed with per-kernel timing off
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
    ms_step = max(ev0.elapsed_time(ev1), wall * 1000) / a.steps
    value = n / (ms_step / 1000.0) / 1e6
    log(f"timed {a.steps} steps: {ms_step:.3f} ms/step")
    # per-kernel times from separate profiled steps
    prof_steps = 3
    K.kpa_profile_enable(True)
    for _ in range(prof_steps):
        pipe.step(rows)
    torch.cuda.synchronize()
    onchip = int(pipe.stats.cpu()[1]) if a.algo == "learned" else 0
    passes = kernel_passes(K, prof_steps, n, PASS_BYTES, entries={"learned_finish": onchip})
    K.kpa_profile_enable(False)

    # Active radix passes: digits that vary inside a window
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
        bytes_per_launch = (24 * n * (active / n_win) / launches if dom == "radix_pass"
                            else PASS_BYTES[dom] * n)
        tr = TRAFFIC.get(("c2", dom))
        traffic = counted_traffic(tr[1], tr[0], tr[2]) if (tr and n == 1 << 28) else None
        roof = roofline(passes, dom, bytes_per_launch, traffic)

    check, cpu = None, None
    if not (a.no_cpu and a.no_check):
        import oracle
        m = min(a.cpu_rows, n)
        host = rows[:m].cpu()
        threads = min(n_win, os.cpu_count() or 1)
        t1 = time.perf_counter()
        g, tk, ts, cs = oracle.window_aggregate(host, LAYOUT32, W, n_win, k=10, n_threads=threads)
        dt = time.perf_counter() - t1
        cpu = {"value": round(m / dt / 1e6, 3), "unit": "Mrec/s", "cores": threads,
               "host_cores": os.cpu_count(), "kind": "oracle",
               "sample": f"first {m} of {n} rows (all their windows), ordered-map keyed "
               f"aggregation + top-10, {dt:.1f} s on {threads} threads"}
        # windows wholly inside the sample: every per-key array and the top-10
        full = [w for w in range(n_win) if (w + 1) * n / n_win + n / 1000 < m]
        hk, hr, hoff, _ = oracle.partition(host, LAYOUT32, W, n_win)
        gs = pipe.gseg.cpu().numpy().view(np.uint64)
        tkg = pipe.top_key.cpu().numpy().view(np.uint64).reshape(n_win, 10)
        tsg = pipe.top_sum.cpu().numpy().view(np.uint64).reshape(n_win, 10)

        def one(w):
            a0, b0 = int(hoff[w]), int(hoff[w + 1])
            return w, oracle.reduce_by_key(hk[a0:b0], hr[a0:b0], host, LAYOUT32)

        with cf.ThreadPoolExecutor(threads) as ex:
            ores = dict(ex.map(one, full))
        ok = True
        for w in full:
            g0, g1 = int(gs[w]), int(gs[w + 1])
            got = [t[g0:g1].cpu().numpy().view(np.uint64) for t in
                   (pipe.gkey, pipe.g["cnt"], pipe.g["sum"], pipe.g["max"])]
            ok = ok and g1 - g0 == int(g[w]) and \
                all(np.array_equal(x, y) for x, y in zip(got, ores[w])) and \
                np.array_equal(tkg[w], tk[w]) and np.array_equal(tsg[w], ts[w])
        check = {"windows_checked": full, "per_key_arrays_and_top10_match_oracle": bool(ok)}
        log(f"oracle sample: {dt:.1f} s on {threads} threads; check {check}")

    return {
        "metric": METRIC, "value": round(value, 2), "unit": "Mrec/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "windowed keyed aggregation: 2^28 32-byte rows, Zipf s=1.1 keys "
                   "over 2^20, 10 tumbling 1 s windows, count/sum/max per key + top-10 by sum",
                   "rows": n, "row_bytes": 32, "windows": n_win, "sort": a.algo},
        "roofline": roof, "cpu_baseline": cpu, "passes": passes, "check": check,
    }


def bench_c3(a):
    """Temporal join + median: two streams of 2^26 32-byte rows, keys uniform
    over 2^24 (one key table for both), values uniform over u64, 10 tumbling
    1 s windows.  One step = partition + sort both streams, lower median per
    key on both, merge-join per window (count, sum of products mod 2^64)."""
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
    K.kpa_profile_enable(True)
    for _ in range(2):
        pipe.step(rows_l, rows_r)
    torch.cuda.synchronize()
    passes = kernel_passes(K, 2, 2 * n, PASS_BYTES)
    K.kpa_profile_enable(False)
    value = 2 * n / (ms_step / 1000.0) / 1e6
    log(f"c3 timed {a.steps} steps: {ms_step:.3f} ms/step")
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
        nk, nm = oracle.median_by_key(rk, rr, hr, LAYOUT32)
        return w, c, s_, (mk, mm), (nk, nm), len(lk) + len(rk)

    with cf.ThreadPoolExecutor(len(checked)) as ex:
        res = list(ex.map(one, checked))
    dt = time.perf_counter() - t1
    m_rows = 0
    for w, c, s_, lmed, rmed, nr in res:
        ok = ok and int(cnt[w]) == c and int(sp[w]) == s_
        for side, med in ((L, lmed), (R, rmed)):
            goff = side["med"]["gseg_off"].cpu().numpy().view(np.uint64)
            a0, b0 = int(goff[w]), int(goff[w + 1])
            ok = ok and np.array_equal(side["med"]["gkey"][a0:b0].cpu().numpy().view(np.uint64),
                                       med[0]) and \
                np.array_equal(side["med"]["gmed"][a0:b0].cpu().numpy().view(np.uint64), med[1])
        m_rows += nr
    check = {"windows_checked": checked, "join_and_both_medians_match_oracle": bool(ok),
             "pairs_per_window": int(cnt[checked[0]])}
    cpu = {"value": round(m_rows / dt / 1e6, 3), "unit": "Mrec/s", "cores": len(checked),
           "host_cores": os.cpu_count(), "kind": "oracle",
           "sample": f"windows {checked} of both streams ({m_rows} rows): ordered-map join + "
           f"median per key, {dt:.1f} s"}
    roof = None
    if "radix_pass" in passes:
        pl = passes["radix_pass"]
        roof = roofline(passes, "radix_pass", 24 * 2 * n * 8 / pl["launches_per_step"])
    return {
        "metric": METRIC, "value": round(value, 2), "unit": "Mrec/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "temporal join + median per key: 2 x 2^26 32-byte rows, keys "
                   "uniform over 2^24, 10 tumbling 1 s windows", "rows": 2 * n, "windows": n_win},
        "roofline": roof, "cpu_baseline": cpu, "passes": passes, "check": check,
    }


def serve_leg(rate, duration, host_rows=False, pool_rows=1 << 25, rate_end=None, wm_lag_s=0.0,
              server_cfg=None, trace=False, allow_fail=False):
    """Serving: Poisson-arriving bundles (sizes log-uniform 2^13..2^20 rows)
    at the offered rate over 16 queries (8 windowed sums, 4 medians, 4 joins
    whose bundles alternate sides), 1 s tumbling windows with origins
    staggered by 1/16 s, a watermark per query every 100 ms of event time.
    Bundles are replayed from pinned pools of pre-generated rows, moved to
    their event time at ingest.  Returns sustained Mrec/s and the p50/p99 of
    window-close-to-result latency.  rate_end: the offered rate grows linearly
    from `rate` to `rate_end` over the run; wm_lag_s: watermarks trail the
    arrivals by that much event time (windows stay open longer); server_cfg:
    overrides of the server configuration; trace: return the monitor's
    samples (placement experiments); allow_fail: a server that stops or
    stalls (memory budget) ends the run with an "error" entry instead of an
    exception."""
    import numpy as np
    import torch

    import datagen
    import paper_1901_01328_amd as P
    from datagen.rows import LAYOUT32
    K = P.load()
    dev = torch.device("cuda:0")
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
    log(f"serving pools of {pool_rows} rows generated in {time.time() - t0:.1f} s")
    W = 10 ** 9
    cfg = dict(budget_bytes=64 << 30, slots=8, rows_in_host=1 if host_rows else 0,
               max_bundle_rows=1 << 20, max_pending=1024)
    cfg.update(server_cfg or {})
    srv = K.Server(**cfg)
    kinds = [K.KPA_Q_SUM] * 8 + [K.KPA_Q_MEDIAN] * 4 + [K.KPA_Q_JOIN] * 4
    qids = [srv.add_query(k, LAYOUT32, W, q * (W // 16)) for q, k in enumerate(kinds)]
    rng = np.random.default_rng(55)
    mean_rows = (2 ** 20 - 2 ** 13) / np.log(2 ** 7)      # log-uniform mean

    def lam_at(t):                                       # bundles per second at time t
        r = rate if rate_end is None else rate + (rate_end - rate) * min(1.0, t / duration)
        return r / mean_rows
    lag = int(wm_lag_s * 1e9)
    side_next = [0] * len(qids)
    n_sub = 0
    last_wm = [0] * len(qids)
    start = time.perf_counter()
    t_next = 0.0
    last_print = 0.0

    def progress(what):
        nonlocal last_print
        now = time.perf_counter() - start
        if now - last_print > 5:
            st = srv.stats()
            log(f"serving {what} t={now:.1f}s bundles={n_sub} closed={st['windows_closed']} "
                f"on_host={st['bundles_on_host']} k_low={st['k_low']:.2f} "
                f"p99={st['p99_ms']:.1f} ms")
            last_print = now

    error = None
    try:
        while True:
            t_next += rng.exponential(1.0 / lam_at(t_next))
            if t_next > duration:
                break
            now = time.perf_counter() - start
            if t_next > now:
                time.sleep(t_next - now)
            nb = int(2 ** rng.uniform(13, 20))
            q = n_sub % len(qids)
            pool = pools[0] if kinds[q] == K.KPA_Q_SUM else pools[1]
            o = int(rng.integers(0, pool_rows - nb))
            side = 0
            if kinds[q] == K.KPA_Q_JOIN:
                side = side_next[q]
                side_next[q] ^= 1
            ev = int(t_next * 1e9) + W        # event time of the bundle (ns)
            # back-pressure: the pending queue is full while the server catches
            # up (a stalled server makes the blocking call report it)
            while True:
                try:
                    srv.submit(qids[q], pool[o:o + nb], side=side, ts_base=ev, ts_lo=0,
                               ts_hi=10 ** 6 - 1, blocking=False)
                    break
                except K.KpaError as e:
                    if "pending queue full (back-pressure)" not in str(e):
                        raise
                    progress("back-pressure")
                    srv.submit(qids[q], pool[o:o + nb], side=side, ts_base=ev, ts_lo=0,
                               ts_hi=10 ** 6 - 1, blocking=True)
                    break
            n_sub += 1
            for qq in range(len(qids)):       # watermarks: every 100 ms of event time
                if ev - lag - last_wm[qq] >= 10 ** 8:
                    srv.watermark(qids[qq], ev - lag)
                    last_wm[qq] = ev - lag
            progress("arrivals")
        end_ev = int(duration * 1e9) + 2 * W + 10 ** 6
        for qq in range(len(qids)):
            srv.watermark(qids[qq], end_ev)
        t_drain = time.perf_counter()
        while True:
            try:
                srv.drain(timeout_ms=2000)
                break
            except K.KpaError as e:
                if e.code != K.KPA_ETIMEOUT or time.perf_counter() - t_drain > 150:
                    raise
                progress("drain")
    except K.KpaError as e:
        if not allow_fail:
            raise
        error = str(e)
        log(f"serving stopped: {error}")
    st = srv.stats()
    res = []
    while True:                            # the results that came out (a failed server
        try:                               # reports its failure once they are taken)
            r = srv.poll(0)
        except K.KpaError:
            break
        if r is None:
            break
        res.append(r)
    tr = srv.trace() if trace else None
    srv.close()
    lat = sorted(r["latency_ms"] for r in res)
    # the closes at the end (after the last watermark) are not steady state
    steady = sorted(r["latency_ms"] for r in res if r["window"] < int(duration) - 1)
    pct = (lambda v, p: v[min(len(v) - 1, int(p * (len(v) - 1) + 0.5))] if v else None)
    extra = {}
    if tr is not None:
        step = max(1, len(tr) // 40)
        extra["trace"] = [{k: (round(v, 4) if isinstance(v, float) else v) for k, v in t.items()}
                          for t in tr[::step]]
        extra["runs_total"] = sum(r["runs"] for r in res)
        extra["runs_from_host"] = sum(r["runs_host"] for r in res)
    if rate_end is not None:
        extra["offered_end_mrec_per_s"] = rate_end / 1e6
    if wm_lag_s:
        extra["watermark_lag_s"] = wm_lag_s
    return {**extra, "offered_mrec_per_s": rate / 1e6, "duration_s": duration, "bundles": n_sub,
            "mrec_per_s": round(st["mrec_per_s"], 2),
            "latency_ms": {"p50": pct(steady, 0.5), "p99": pct(steady, 0.99),
                           "max": lat[-1] if lat else None, "windows": len(steady)},
            "rows_in_host": bool(host_rows), "budget_gib": cfg["budget_bytes"] / 2 ** 30,
            **({"error": error} if error else {}),
            "queries": "8 sum + 4 median + 4 join, 1 s windows, watermark every 100 ms",
            "server": st}


def bench_adapt(a):
    """The paper's two adaptation experiments (Sec. 7.3), with the capacity
    tier a pinned host pool and a device budget smaller than the open
    windows' KPAs at the higher load: (a) the offered rate ramps from 200M to
    1G rec/s over the run; (b) watermarks trail the arrivals by 3 s at 400M
    rec/s, so windows stay open and hold their KPAs longer.  Balanced
    placement (impact tags and the demand balance knob) against all-device
    placement on the same input; a run whose server stalls or stops for
    memory reports it under "error"."""
    runs = {}
    base = dict(budget_bytes=24 << 30, reserve_pct=40, host_pool_bytes=48 << 30, monitor_ms=10,
                target_delay_ms=1000.0, rows_in_host=1)
    for name, kw in (("rate_ramp", dict(rate=200e6, rate_end=1.0e9)),
                     ("delayed_watermarks", dict(rate=400e6, wm_lag_s=3.0))):
        for placement in ("balanced", "device"):
            import paper_1901_01328_amd as P
            K = P.load()
            cfg = dict(base, placement=K.KPA_PLACE_BALANCED if placement == "balanced"
                       else K.KPA_PLACE_DEVICE)
            if placement == "device":
                cfg.pop("host_pool_bytes")
            log(f"adapt {name} {placement}")
            r = serve_leg(duration=a.duration, host_rows=True, server_cfg=cfg,
                          trace=placement == "balanced", allow_fail=True, **kw)
            runs.setdefault(name, {})[placement] = r
    return {"metric": METRIC, "workload": "adaptation: serving with a 24 GiB device budget "
            "(40% close reserve), a 48 GiB pinned host pool, rows kept on the host",
            "runs": runs}


def bench_ads(a):
    """The paper's pipeline example on KPAs (Filter by event type, external
    join ad -> campaign by key update and write-back, KeySwap to time,
    Partition into 1 s windows, KeySwap to the campaign, sort, count) over
    `--rows` synthetic ad events; every window's per-campaign counts are
    compared with their definition counted on the host."""
    import numpy as np
    import torch

    import datagen
    from paper_1901_01328_amd.pipeline import AdPipeline
    n, W, n_win = a.rows, 10 ** 9, 10
    dev = torch.device("cuda:0")
    rows = datagen.gen_ysb(n, device=dev)
    tk, tv = datagen.ysb_tables(device=dev)
    pipe = AdPipeline(n, tk, tv, W, n_win)
    for _ in range(a.warmup):
        info = pipe.step(rows)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        info = pipe.step(rows)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000 / a.steps
    log(f"ads: {a.steps} steps, {ms:.3f} ms/step, {info}")
    check = None
    if not a.no_check:
        h = rows.cpu().numpy().view(np.uint64)
        keep = h[:, 1] == np.uint64(datagen.YSB_VIEW)
        ads, ts = h[keep, 0], h[keep, 2]
        tkh, tvh = tk.cpu().numpy().view(np.uint64), tv.cpu().numpy().view(np.uint64)
        pos = np.minimum(np.searchsorted(tkh, ads), len(tkh) - 1)
        camp = np.where(tkh[pos] == ads, tvh[pos], ads)
        win = ts // np.uint64(W)
        gs = pipe.gseg.cpu().numpy().view(np.uint64)
        gk, gc = pipe.gkey.cpu().numpy().view(np.uint64), pipe.gcnt.cpu().numpy().view(np.uint64)
        ok = True
        for w in range(n_win):
            ks, cs = np.unique(camp[win == np.uint64(w)], return_counts=True)
            g0, g1 = int(gs[w]), int(gs[w + 1])
            ok = ok and np.array_equal(gk[g0:g1], ks) and np.array_equal(gc[g0:g1], cs)
        check = {"windows_checked": n_win, "per_campaign_counts_match_definition": bool(ok)}
        log(f"ads check {check}")
    return {"metric": METRIC, "value": round(n / (ms / 1000) / 1e6, 2), "unit": "Mrec/s",
            "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms, 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
            "data": "synthetic",
            "config": {"workload": f"ad-event pipeline: {n} 32-byte rows, 1000 campaigns x 10 "
                       "ads, filter views, external join by key update + write-back, 10 x 1 s "
                       "windows, count per campaign", "survivors": info["survivors"]},
            "check": check}


def bench_models(a):
    """Where the learned sort's models come from: 8 substream windows of 2^22
    keys shaped like C4's (substreams 0, 512, ..., 3584: rank-Zipf keys whose
    exponent grows with the substream); epoch 0's sorted windows give (a) a
    direct PWL fit per window and (b) the monotone MLP trained on the GPU per
    window (4096 samples, 400 Adam steps, lr 1e-2) and distilled to PWL
    knots.  Epoch 1's windows are then sorted by radix and by the learned
    sort with each model set (identical output checked); reported: time to
    build each model set, sort times and the learned path's counters."""
    import numpy as np
    import torch

    import datagen
    import paper_1901_01328_amd as P
    K = P.load()
    dev = torch.device("cuda:0")
    subs, n = list(range(0, 4096, 512)), 1 << 22
    off = torch.tensor([w * n for w in range(len(subs) + 1)], dtype=torch.int64, device=dev)

    def keys(epoch):
        return torch.cat([datagen.gen_c4_window(j, epoch, n, device=dev)[:, 0] for j in subs])

    def timed(fn, reps=5):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            out = fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps, out

    k0 = keys(0)
    sk0, _ = K.kpa_sort_segmented(k0, None, off)
    ms_pwl, m_pwl = timed(lambda: K.kpa_pwl_fit(sk0, off, 1024), reps=3)
    # one network per window, its random start drawn here and passed in
    from datagen.rows import uniform_f64
    u = uniform_f64(datagen.splitmix64(77, 1, torch.arange(
        len(subs) * K.KPA_MLP_PARAMS, dtype=torch.int64, device=dev))).float()
    m_mlp = K.new_models(len(subs), dev)
    mb = K.PWL_MODEL_BYTES
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = []
    for w in range(len(subs)):
        model = m_mlp[w * mb:(w + 1) * mb]
        x, y = K.kpa_mlp_training_set(sk0[w * n:(w + 1) * n], 4096, model)
        p = K.kpa_mlp_init(u[w * K.KPA_MLP_PARAMS:(w + 1) * K.KPA_MLP_PARAMS].contiguous())
        mm, vv = torch.zeros_like(p), torch.zeros_like(p)
        losses.append(K.kpa_mlp_train(p, mm, vv, x, y, 1, 400, lr=1e-2))
        K.kpa_mlp_to_pwl(p, model, 1024)
    torch.cuda.synchronize()
    ms_mlp = (time.perf_counter() - t0) * 1000
    log(f"models: pwl fit {ms_pwl:.3f} ms, mlp train+distill {ms_mlp:.1f} ms")
    k1 = keys(1)
    res = {}
    ms_r, (rk, rr) = timed(lambda: K.kpa_sort_segmented(k1, None, off))
    res["radix"] = {"sort_ms": round(ms_r, 3)}
    for name, models in (("learned_pwl", m_pwl), ("learned_mlp", m_mlp)):
        st = K.new_sort_stats(dev)
        ms_l, (lk, lr) = timed(lambda: K.kpa_sort_segmented(
            k1, None, off, algo=K.KPA_SORT_LEARNED, models=models, stats=st))
        s = st.cpu().numpy().tolist()
        same = bool(torch.equal(lk, rk) and torch.equal(lr, rr))
        res[name] = {"sort_ms": round(ms_l, 3), "speedup_vs_radix": round(ms_r / ms_l, 3),
                     "finished_on_chip": s[1], "single_key_entries": s[2],
                     "fallback_entries": s[3], "order_violations": s[5],
                     "identical_to_radix": same}
        log(f"{name}: {res[name]}")
    return {"metric": METRIC, "workload": f"{len(subs)} windows of {n} keys (C4 substreams "
            f"{subs[0]}..{subs[-1]}), epoch 0 -> models, epoch 1 sorted",
            "model_build_ms": {"pwl_fit": round(ms_pwl, 3), "mlp_train_distill": round(ms_mlp, 1)},
            "mlp_final_loss": [round(float(l.item()), 6) for l in losses], "sorts": res}


def bench_c5(a):
    # Beyond what the budget holds (a 1 s window of rows above 64 GiB) the
    # server stops admitting and says so; the line then reports the rate
    # sustained until then under "error" and the run exits with status 1.
    s = serve_leg(a.rate, a.duration, host_rows=a.host_rows, allow_fail=True)
    return {
        "metric": METRIC, "value": s["mrec_per_s"], "unit": "Mrec/s", "n_gpus": 1,
        "steps": s["bundles"], "warmup": 0, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "serving: Poisson bundles of 2^13..2^20 32-byte rows at "
                   f"{a.rate / 1e6:.0f} M rec/s offered, 8 sum + 4 median + 4 join queries, "
                   "1 s windows, watermark every 100 ms", "duration_s": a.duration,
                   "rows_in_host": bool(a.host_rows), "budget_gib": 64},
        "latency_ms": s["latency_ms"], "server": s["server"], "roofline": None,
        "cpu_baseline": None, **({"error": s["error"]} if "error" in s else {}),
    }


if __name__ == "__main__":
    main()
