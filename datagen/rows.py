"""Counter-based SplitMix64 streams and row packing for the synthetic workloads.

Every value is a pure function of (seed, stream id, element index), so any
slice of a workload can be regenerated on its own, on the CPU or on a GPU, with
identical bits (integer arithmetic only, plus float64 comparisons against a
host-built table for Zipf ranks).

SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): state_i = key + (i+1)*GOLDEN,
output = mix(state_i) with the 64-bit finalizer below.

Row layouts follow the paper's benchmark records: numeric 64-bit columns for
key, value and event timestamp (Sec. 6, Benchmarks).  The small workload packs
{u64 key, u32 value, u32 timestamp} into 16 bytes; the others use 32-byte rows
{u64 key, u64 value, u64 timestamp, u64 pad}.
"""
from __future__ import annotations

import functools
import math
from dataclasses import dataclass

import numpy as np
import torch

GOLDEN = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB


def _s64(c: int) -> int:
    """Reinterpret an unsigned 64-bit constant as a signed int64."""
    c &= (1 << 64) - 1
    return c - (1 << 64) if c >= (1 << 63) else c


def _srl(x: torch.Tensor, k: int) -> torch.Tensor:
    """Logical right shift of an int64 tensor holding u64 bit patterns."""
    return (x >> k) & ((1 << (64 - k)) - 1)


def mix64(z: torch.Tensor) -> torch.Tensor:
    """SplitMix64 finalizer (a bijection on 64-bit words)."""
    z = (z ^ _srl(z, 30)) * _s64(_M1)
    z = (z ^ _srl(z, 27)) * _s64(_M2)
    return z ^ _srl(z, 31)


def mix64_int(z: int) -> int:
    """Python-int version of ``mix64`` (used for stream keys and tests)."""
    m = (1 << 64) - 1
    z &= m
    z = ((z ^ (z >> 30)) * _M1) & m
    z = ((z ^ (z >> 27)) * _M2) & m
    return z ^ (z >> 31)


def stream_key(seed: int, stream: int) -> int:
    return mix64_int(((seed & 0xFFFFFFFFFFFF) << 16) ^ (stream & 0xFFFF) ^ 0x5851F42D4C957F2D)


def splitmix64(seed: int, stream: int, idx: torch.Tensor) -> torch.Tensor:
    """u64 bit patterns (as int64) of element ``idx`` of stream (seed, stream)."""
    key = _s64(stream_key(seed, stream))
    return mix64(key + (idx + 1) * _s64(GOLDEN))


def uniform_int(u: torch.Tensor, m: int) -> torch.Tensor:
    """Map u64 words to integers in [0, m) for 0 < m <= 2^31 (multiply-high)."""
    assert 0 < m <= (1 << 31)
    return (_srl(u, 32) * m) >> 32


def uniform_u64(u: torch.Tensor) -> torch.Tensor:
    return u


def uniform_f64(u: torch.Tensor) -> torch.Tensor:
    """u64 words -> float64 in [0, 1) with 53 random bits (exact)."""
    return _srl(u, 11).to(torch.float64) * (2.0 ** -53)


@functools.lru_cache(maxsize=64)
def _zipf_cdf_np(s: float, k: int) -> np.ndarray:
    r = np.arange(1, k + 1, dtype=np.float64)
    w = r ** (-s)
    c = np.cumsum(w)  # sequential float64 sum on the host: reproducible
    return c / c[-1]


def zipf_cdf_table(s: float, k: int, device="cpu") -> torch.Tensor:
    return torch.from_numpy(_zipf_cdf_np(float(s), int(k))).to(device)


def zipf_ranks(u: torch.Tensor, s: float, k: int) -> torch.Tensor:
    """Zipf(s, k) ranks in [1, k] by inversion of the host-built CDF table."""
    cdf = zipf_cdf_table(s, k, u.device)
    x = uniform_f64(u)
    r = torch.searchsorted(cdf, x, right=True) + 1
    return torch.clamp(r, max=k)


def key_table(k: int, seed: int, device="cpu") -> torch.Tensor:
    """Distinct pseudo-random 64-bit keys: table[i] = mix64(i xor seed)."""
    i = torch.arange(k, dtype=torch.int64, device=device)
    return mix64(i ^ _s64(seed))


@dataclass(frozen=True)
class RowLayout:
    row_bytes: int
    key_off: int
    val_off: int
    val_w: int
    ts_off: int
    ts_w: int


LAYOUT16 = RowLayout(16, 0, 8, 4, 12, 4)
LAYOUT32 = RowLayout(32, 0, 8, 8, 16, 8)


def pack_rows16(key, val, ts) -> torch.Tensor:
    """16-byte rows {u64 key, u32 val, u32 ts} as an int64 [n, 2] tensor."""
    out = torch.empty((key.shape[0], 2), dtype=torch.int64, device=key.device)
    out[:, 0] = key
    out[:, 1] = (val & 0xFFFFFFFF) | ((ts & 0xFFFFFFFF) << 32)
    return out


def pack_rows32(key, val, ts, pad) -> torch.Tensor:
    """32-byte rows {u64 key, u64 val, u64 ts, u64 pad} as an int64 [n, 4] tensor."""
    return torch.stack([key, val, ts, pad], dim=1).contiguous()


# --------------------------------------------------------------------------
# Workloads.  Stream ids: 1 key draw, 2 value, 3 timestamp jitter.
# --------------------------------------------------------------------------

def gen_c1(n: int = 1 << 20, seed: int = 1, device="cpu", n_keys: int = 1000):
    """Small plain workload: 16-byte rows, keys uniform over ``n_keys`` distinct
    64-bit keys, values uniform [0,1000), timestamps (ms) increasing over 1 s."""
    i = torch.arange(n, dtype=torch.int64, device=device)
    table = key_table(n_keys, seed ^ 0xC1, device)
    key = table[uniform_int(splitmix64(seed, 1, i), n_keys)]
    val = uniform_int(splitmix64(seed, 2, i), 1000)
    ts = (i * 1000) // max(n, 1)
    return pack_rows16(key, val, ts)


def _jittered_ts(i, n, span, jitter, seed, device_stream=3):
    base = (i * span) // max(n, 1)
    j = uniform_int(splitmix64(seed, device_stream, i), 2 * jitter + 1) - jitter
    return torch.clamp(base + j, 0, span - 1)


def gen_c2(n: int = 1 << 28, seed: int = 2, device="cpu", n_keys: int = 1 << 20,
           zipf_s: float = 1.1, span_ns: int = 10 ** 10, chunk: int = 1 << 24,
           out: torch.Tensor | None = None):
    """Windowed aggregation workload: 32-byte rows, Zipf(s) keys over ``n_keys``
    distinct keys, values uniform [0, 2^20), ns timestamps over ``span_ns`` with
    +-1 ms bounded disorder, pad = mix64(row index)."""
    if out is None:
        out = torch.empty((n, 4), dtype=torch.int64, device=device)
    table = key_table(n_keys, seed ^ 0xC2, out.device)
    jitter = 10 ** 6 if span_ns >= 10 ** 9 else max(1, span_ns // 10000)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        i = torch.arange(s, e, dtype=torch.int64, device=out.device)
        r = zipf_ranks(splitmix64(seed, 1, i), zipf_s, n_keys)
        out[s:e, 0] = table[r - 1]
        out[s:e, 1] = _srl(splitmix64(seed, 2, i), 44)
        out[s:e, 2] = _jittered_ts(i, n, span_ns, jitter, seed)
        out[s:e, 3] = mix64(i)
    return out


def gen_c3(n: int = 1 << 26, seed: int = 3, side: int = 0, device="cpu",
           n_keys: int = 1 << 24, span_ns: int = 10 ** 10, chunk: int = 1 << 24):
    """One side of the temporal-join workload: keys uniform over ``n_keys``
    distinct keys (one table for both sides), values uniform over all of u64."""
    out = torch.empty((n, 4), dtype=torch.int64, device=device)
    table = key_table(n_keys, seed ^ 0xC3, device)
    sseed = seed * 2 + side + 1
    jitter = 10 ** 6 if span_ns >= 10 ** 9 else max(1, span_ns // 10000)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        i = torch.arange(s, e, dtype=torch.int64, device=device)
        out[s:e, 0] = table[uniform_int(splitmix64(sseed, 1, i), n_keys)]
        out[s:e, 1] = splitmix64(sseed, 2, i)
        out[s:e, 2] = _jittered_ts(i, n, span_ns, jitter, sseed)
        out[s:e, 3] = mix64(i ^ _s64(sseed << 40))
    return out


# Advertising-event stream shaped like the Yahoo streaming benchmark's
# (synthetic: no item of that benchmark is used).  32-byte rows
# {ad_id, event_type, ts, campaign slot}; event types 0 (view), 1 (click),
# 2 (purchase) uniform; ads uniform over n_camps * ads_per_camp ad keys plus
# n_unknown keys absent from the ad table; the campaign slot holds
# mix64(row index) until a pipeline writes a campaign there.
YSB_VIEW = 0
YSB_COLS = {"ad_id": 0, "event_type": 8, "ts": 16, "campaign": 24}
LAYOUT_YSB = RowLayout(32, 0, 8, 8, 16, 8)   # key ad_id, value event_type, ts


def ysb_tables(n_camps: int = 1000, ads_per_camp: int = 10, seed: int = 6, device="cpu"):
    """(ad keys ascending, their campaign keys): the external key-value table."""
    n_ads = n_camps * ads_per_camp
    ads = key_table(n_ads, seed ^ 0xAD, device)
    camps = key_table(n_camps, seed ^ 0xCA, device)[torch.arange(n_ads, device=device)
                                                       // ads_per_camp]
    # the store is looked up by ad key: hand it over in ascending key order
    idx = torch.from_numpy(np.argsort(ads.cpu().numpy().view(np.uint64), kind="stable"))
    idx = idx.to(device)
    return ads[idx], camps[idx]


def gen_ysb(n: int, seed: int = 6, device="cpu", n_camps: int = 1000, ads_per_camp: int = 10,
            n_unknown: int = 16, span_ns: int = 10 ** 10, chunk: int = 1 << 24,
            out: torch.Tensor | None = None):
    if out is None:
        out = torch.empty((n, 4), dtype=torch.int64, device=device)
    n_ads = n_camps * ads_per_camp
    ads = key_table(n_ads, seed ^ 0xAD, out.device)
    unknown = key_table(n_unknown, seed ^ 0x0B, out.device) if n_unknown else ads[:0]
    pool = torch.cat([ads, unknown])
    jitter = 10 ** 6 if span_ns >= 10 ** 9 else max(1, span_ns // 10000)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        i = torch.arange(s, e, dtype=torch.int64, device=out.device)
        out[s:e, 0] = pool[uniform_int(splitmix64(seed, 1, i), pool.numel())]
        out[s:e, 1] = uniform_int(splitmix64(seed, 2, i), 3)
        out[s:e, 2] = _jittered_ts(i, n, span_ns, jitter, seed)
        out[s:e, 3] = mix64(i)
    return out


def c4_window_sizes(n_windows: int = 4096, seed: int = 4, lo_log2: int = 10,
                    hi_log2: int = 22) -> np.ndarray:
    """Substream window sizes, log-uniform over [2^lo, 2^hi): host-side metadata."""
    u = uniform_f64(splitmix64(seed, 7, torch.arange(n_windows, dtype=torch.int64))).numpy()
    return np.floor(np.exp2(lo_log2 + (hi_log2 - lo_log2) * u)).astype(np.int64)


def c4_zipf_s(j: int, epoch: int, n_windows: int = 4096) -> float:
    return min(1.4, 0.8 + 0.6 * j / max(n_windows - 1, 1) + 0.02 * epoch)


def zipf_cdf_table_torch(s: float, k: int, device) -> torch.Tensor:
    """Zipf(s, k) CDF built with torch on ``device`` (float64; the summation
    order is the device's, so the table may differ from the host-built one in
    the last bits).  Used where thousands of distinct exponents are needed."""
    r = torch.arange(1, k + 1, dtype=torch.float64, device=device)
    c = torch.cumsum(r.pow(-float(s)), 0)
    return c / c[-1]


def gen_c4_window(j: int, epoch: int, n: int, seed: int = 4, device="cpu",
                  n_windows: int = 4096, control: bool = False, k: int = 1 << 20,
                  out: torch.Tensor | None = None):
    """Rows of substream ``j`` in ``epoch``: rank-ordered Zipf keys
    o + (r-1)*2^12 with o = j*2^40 + epoch*2^26 (drifting skew and offset), or
    the control variant o + (mix64(r) >> 32).  Values uniform [0, 2^20),
    timestamps spread over one 1 s window, pad = mix64(i).  The Zipf table is
    built on ``device``."""
    dev = out.device if out is not None else device
    i = torch.arange(n, dtype=torch.int64, device=dev)
    sseed = (seed << 20) ^ (j << 4) ^ epoch
    s = c4_zipf_s(j, epoch, n_windows)
    cdf = zipf_cdf_table_torch(s, k, dev)
    r = torch.clamp(torch.searchsorted(cdf, uniform_f64(splitmix64(sseed, 1, i)), right=True) + 1,
                    max=k)
    o = (j << 40) + (epoch << 26)
    if out is None:
        out = torch.empty((n, 4), dtype=torch.int64, device=dev)
    key = o + _srl(mix64(r), 32) if control else o + (r - 1) * (1 << 12)
    # one interleaving write (no strided column copies)
    torch.stack([key, _srl(splitmix64(sseed, 2, i), 44), (i * 10 ** 9) // max(n, 1), mix64(i)],
                dim=1, out=out)
    return out


def gen_c4(epoch: int, sizes: np.ndarray, seed: int = 4, device="cpu",
           out: torch.Tensor | None = None, control: bool = False):
    """All substreams' windows of one epoch back to back (substream j's rows at
    [sum(sizes[:j]), sum(sizes[:j+1])))."""
    total = int(np.sum(sizes))
    if out is None:
        out = torch.empty((total, 4), dtype=torch.int64, device=device)
    a = 0
    for j, n in enumerate(sizes):
        n = int(n)
        if n:
            gen_c4_window(j, epoch, n, seed, n_windows=len(sizes), control=control,
                          out=out[a:a + n])
        a += n
    return out


def as_u64(t: torch.Tensor) -> np.ndarray:
    """View an int64 tensor's bits as a uint64 numpy array (host)."""
    return t.detach().cpu().numpy().view(np.uint64)


def log2ceil(x: int) -> int:
    return 0 if x <= 1 else int(math.ceil(math.log2(x)))
