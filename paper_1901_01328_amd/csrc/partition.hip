// Extract fused with windowing (Sec. 4.2 "Windowing": Partition on the
// timestamp column, the window length being the range of each partition).
//
// Two passes over the rows:
//   1. histogram of window ids (plus out-of-range rows) into global counters,
//      one histogram per chunk of 2^29 rows;
//   2. a single onesweep scatter pass with digit = window id, which reads the
//      key and timestamp of each row and writes (key, rid) into its window.
// The scatter is stable, so each window lists its rows in arrival order.
// The look-back words hold 30-bit counts, so the tiles of each chunk form
// their own look-back chain and start from the chunk's window offsets (the
// windows' starts plus the rows of earlier chunks): any n below 2^32 works.
//
// The same kernels partition a KPA whose resident key is the timestamp
// (rows = the key array read as 8-byte rows, rids taken from the KPA).
#include "digit_sort.hpp"

namespace kpa {

constexpr u32 PART_HIST_ROWS = 1u << 16;  // most rows per histogram workgroup
constexpr u32 PART_CHUNK_LOG2 = 29;       // rows per look-back chain: 2^29
constexpr u32 PART_CHUNK_TILES = (1u << PART_CHUNK_LOG2) / TILE;
static_assert(((1u << PART_CHUNK_LOG2) % PART_HIST_ROWS) == 0, "histogram blocks inside chunks");

struct WinParams {
  u64 origin;
  u64 win_len;
  u64 limit;  // n_win * win_len (exclusive end of the last window, relative)
  double inv; // 1 / win_len
  float inv_f;  // 1 / win_len in single precision
  u32 n_win;
  u32 fast;   // (n_win + 1) * win_len fits in 64 bits: quotient by estimate + correction
};

// Window starts of a workgroup's scatter: bound[w] = origin + w*win_len for
// w = 0..n_win, saturated at 2^64-1 (nondecreasing).  Filled by all threads;
// the caller synchronizes.
__device__ __forceinline__ void fill_bounds(u64* bound, const WinParams& p) {
  for (u32 w = threadIdx.x; w <= p.n_win; w += blockDim.x) {
    u64 off, b;
    const bool ovf = __builtin_mul_overflow((u64)w, p.win_len, &off) ||
                     __builtin_add_overflow(p.origin, off, &b);
    bound[w] = ovf ? ~0ull : b;
  }
}

// Window of a timestamp from the table: a single-precision estimate of
// (ts - origin) / win_len (its relative error is below 2^-21, so for fewer than
// 256 windows it is within one of the quotient), corrected by comparing ts
// with the two window starts around it.  Equals the integer quotient whenever
// the quotient is below n_win; false for timestamps outside all windows.
__device__ __forceinline__ bool window_of_table(u64 ts, const u64* bound, const WinParams& p,
                                                u32& w) {
  if (ts < bound[0] || ts >= bound[p.n_win]) return false;
  u32 q = (u32)((float)(ts - p.origin) * p.inv_f);
  q = q < p.n_win - 1 ? q : p.n_win - 1;
  if (ts < bound[q]) --q;
  else if (ts >= bound[q + 1]) ++q;
  w = q;
  return true;
}

// Window of a timestamp, exactly as the integer quotient (ts - origin) / win_len.
__device__ __forceinline__ bool window_of(u64 ts, const WinParams& p, u32& w) {
  if (ts < p.origin) return false;
  const u64 x = ts - p.origin;
  if (p.fast) {
    if (x >= p.limit) return false;
    // The double-precision estimate is within one of the true quotient (which
    // is below 256); fix it with exact integer products.
    u64 q = (u64)((double)x * p.inv);
    if (q * p.win_len > x) --q;
    else if ((q + 1) * p.win_len <= x) ++q;
    w = (u32)q;
    return true;
  }
  const u64 q = x / p.win_len;
  if (q >= p.n_win) return false;
  w = (u32)q;
  return true;
}

__device__ __forceinline__ u64 load_ts(const unsigned char* row, u32 ts_off, u32 ts_w) {
  return ts_w == 8 ? *reinterpret_cast<const u64*>(row + ts_off)
                   : (u64)*reinterpret_cast<const u32*>(row + ts_off);
}

constexpr int PART_HIST_U = 16;  // rows per thread in flight


// Window histogram: each thread keeps PART_HIST_U row loads in flight; rows
// of one window are counted per wave with one LDS atomic (consecutive rows
// mostly share a window); the optional value column is copied out on the way.
__global__ void __launch_bounds__(BLOCK) k_part_hist(const unsigned char* __restrict__ rows,
                                                     u64 n, u32 row_bytes, u32 ts_off, u32 ts_w,
                                                     WinParams wp, u32* __restrict__ counts,
                                                     u32 val_off, u32 val_w,
                                                     u64* __restrict__ out_vals, u32 rpb) {
  __shared__ u32 h[WAVES][RADIX + 1];
  const u32 tid = threadIdx.x;
  const u32 w = tid >> 6;
  for (u32 i = tid; i < WAVES * (RADIX + 1); i += BLOCK) (&h[0][0])[i] = 0;
  __syncthreads();
  const u64 r0 = (u64)blockIdx.x * rpb;
  const u64 r1 = min(n, r0 + rpb);
  counts += (r0 >> PART_CHUNK_LOG2) * (RADIX + 1);
  for (u64 b = r0; b < r1; b += (u64)BLOCK * PART_HIST_U) {
    u64 ts[PART_HIST_U], vv[PART_HIST_U];
#pragma unroll
    for (int j = 0; j < PART_HIST_U; ++j) {
      const u64 i = b + tid + (u64)j * BLOCK;
      ts[j] = 0;
      vv[j] = 0;
      if (i < r1) {
        const unsigned char* row = rows + i * row_bytes;
        ts[j] = load_ts(row, ts_off, ts_w);
        if (out_vals) vv[j] = load_ts(row, val_off, val_w);
      }
    }
#pragma unroll
    for (int j = 0; j < PART_HIST_U; ++j) {
      const u64 i = b + tid + (u64)j * BLOCK;
      const bool v = i < r1;
      u32 win;
      const u32 d = v && window_of(ts[j], wp, win) ? win : (u32)RADIX;
      wave_hist_add(h[w], d, v);
      if (v && out_vals) out_vals[i] = vv[j];
    }
  }
  __syncthreads();
  for (u32 d = tid; d <= RADIX; d += BLOCK) {
    u32 c = 0;
#pragma unroll
    for (int ww = 0; ww < WAVES; ++ww) c += h[ww][d];
    if (c && (d < wp.n_win || d == RADIX)) atomicAdd(&counts[d], c);
  }
}

// counts (per chunk) -> exclusive window offsets (u64 for the caller) and,
// per chunk, where each window's rows of that chunk begin (u32, the
// scatter's bases: n < 2^32).
__global__ void __launch_bounds__(BLOCK) k_part_scan(const u32* __restrict__ counts,
                                                     u32 n_chunks, u32 n_win,
                                                     u32* __restrict__ woff,
                                                     u64* __restrict__ win_off,
                                                     u64* __restrict__ oob) {
  __shared__ u64 sc[WAVES + 1];
  const u32 tid = threadIdx.x, lane = __lane_id(), w = tid >> 6;
  u64 c = 0;
  if (tid < n_win)
    for (u32 k = 0; k < n_chunks; ++k) c += counts[k * (RADIX + 1) + tid];
  u64 incl = c;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const u64 t = __shfl_up(incl, o, 64);
    if (lane >= (u32)o) incl += t;
  }
  if (lane == 63) sc[w] = incl;
  __syncthreads();
  u64 ex = incl - c, tot = 0;
  for (u32 i = 0; i < WAVES; ++i) {
    if (i < w) ex += sc[i];
    tot += sc[i];
  }
  if (tid < n_win) {
    win_off[tid] = ex;
    u64 run = ex;
    for (u32 k = 0; k < n_chunks; ++k) {
      woff[k * RADIX + tid] = (u32)run;
      run += counts[k * (RADIX + 1) + tid];
    }
  }
  if (tid == 0) {
    win_off[n_win] = tot;
    u64 o = 0;
    for (u32 k = 0; k < n_chunks; ++k) o += counts[k * (RADIX + 1) + RADIX];
    *oob = o;
  }
}

// The scatter: persistent workgroups of PASS_WAVES waves (two per CU) claim
// tiles in order.  (Prefetching the next tile's rows during the look-back, as
// the sort passes do, needs the keys and timestamps of two tiles in registers
// here and spills.)
__global__ void __launch_bounds__(PASS_THREADS, PASS_WAVES / 2)
    k_part_pass(const unsigned char* __restrict__ rows, u64 n, u32 row_bytes, u32 key_off,
                u32 ts_off, u32 ts_w, WinParams wp, u32 rid_base,
                const u32* __restrict__ rids_in, const u32* __restrict__ woff,
                u32 n_tiles, u32* __restrict__ status, u32* __restrict__ counter,
                u64* __restrict__ keys_out, u32* __restrict__ rids_out) {
  __shared__ OnesweepSmemT<PASS_WAVES> sm;
  __shared__ u64 bound[RADIX + 1];
  const u32 tid = threadIdx.x;
  fill_bounds(bound, wp);  // the claim below synchronizes
  auto claim = [&]() -> u32 {
    __syncthreads();
    if (tid == 0) sm.tile = atomicAdd(counter, 1u);
    __syncthreads();
    return sm.tile;
  };
  u64 kk[PASS_ITEMS], tt[PASS_ITEMS];
  u32 rr[PASS_ITEMS], dd[PASS_ITEMS];
  u32 dpk[(PASS_ITEMS + 3) / 4];  // window digits, four to a word
  // Row loads of a tile: timestamps, then (separately) keys.
  auto load_ts_of = [&](u32 tile) {
    const u64 base = (u64)tile * TILE;
#pragma unroll
    for (int j = 0; j < PASS_ITEMS; ++j) {
      const u64 e = base + tile_offset_t<PASS_WAVES>(j);
      tt[j] = e < n ? load_ts(rows + e * row_bytes, ts_off, ts_w) : 0ull;
    }
  };
  auto load_keys_of = [&](u32 tile) {
    const u64 base = (u64)tile * TILE;
#pragma unroll
    for (int j = 0; j < PASS_ITEMS; ++j) {
      const u64 e = base + tile_offset_t<PASS_WAVES>(j);
      kk[j] = e < n ? *reinterpret_cast<const u64*>(rows + e * row_bytes + key_off) : 0ull;
    }
  };
  // Window digits (packed into dpk) from the loaded timestamps.
  auto digits = [&](u32 tile) -> u32 {
    const u64 base = (u64)tile * TILE;
    u32 valid = 0;
#pragma unroll
    for (int i = 0; i < (PASS_ITEMS + 3) / 4; ++i) dpk[i] = 0;
#pragma unroll
    for (int j = 0; j < PASS_ITEMS; ++j) {
      const u64 e = base + tile_offset_t<PASS_WAVES>(j);
      u32 win;
      if (e < n && window_of_table(tt[j], bound, wp, win)) {
        dpk[j >> 2] |= win << (8 * (j & 3));
        valid |= 1u << j;
      }
    }
    return valid;
  };
  u32 tile = claim();
  if (tile >= n_tiles) return;
  load_ts_of(tile);
  load_keys_of(tile);
  u32 valid = digits(tile);
  while (true) {
    const u32 chunk = tile / PART_CHUNK_TILES, t_in = tile % PART_CHUNK_TILES;
    const u64 my_base = tid < wp.n_win ? (u64)woff[chunk * RADIX + tid] : 0ull;
#pragma unroll
    for (int j = 0; j < PASS_ITEMS; ++j) {
      const u64 e = (u64)tile * TILE + tile_offset_t<PASS_WAVES>(j);
      rr[j] = rids_in ? (e < n ? rids_in[e] : 0u) : rid_base + (u32)e;
      dd[j] = (dpk[j >> 2] >> (8 * (j & 3))) & 255u;
    }
    u32 tile_count;
    const u32 cnt_d = onesweep_rank_stage(sm, kk, rr, dd, valid, status, tile, t_in, &tile_count);
    onesweep_lookback_write(sm, status, tile, t_in, cnt_d, tile_count, my_base, keys_out,
                            rids_out);
    const u32 next = claim();
    if (next >= n_tiles) return;
    load_ts_of(next);
    load_keys_of(next);
    const u32 nvalid = digits(next);
    tile = next;
    valid = nvalid;
  }
}

struct PartWs {
  u32* counts;  // per chunk: RADIX + 1 (windows, then out-of-range rows)
  u32* woff;    // per chunk: RADIX window bases
  u32* counter;
  u32* status;
  u64 n_tiles;
  u32 n_chunks;
};

static void part_plan(u64 n, Carver& c, PartWs* w) {
  w->n_tiles = ceil_div(n ? n : 1, TILE);
  w->n_chunks = (u32)ceil_div(n ? n : 1, 1ull << PART_CHUNK_LOG2);
  w->counts = c.take<u32>((u64)w->n_chunks * (RADIX + 1));
  w->woff = c.take<u32>((u64)w->n_chunks * RADIX);
  w->counter = c.take<u32>(1);
  w->status = c.take<u32>(w->n_tiles * RADIX);
}

static kpa_status part_launch(const unsigned char* r, u64 n, u32 row_bytes, u32 key_off,
                              u32 ts_off, u32 ts_w, u32 val_off, u32 val_w, u64 win_len,
                              u64 win_origin, u32 n_win, u32 rid_base, const u32* rids_in,
                              u64* out_keys, u32* out_rids, u64* out_vals, u64* out_win_off,
                              u64* out_oob, const PartWs& w, hipStream_t stream) {
  WinParams wp;
  wp.origin = win_origin;
  wp.win_len = win_len;
  wp.n_win = n_win;
  unsigned __int128 lim = (unsigned __int128)win_len * (n_win + 1);
  wp.fast = lim < ((unsigned __int128)1 << 64) ? 1u : 0u;
  wp.limit = wp.fast ? win_len * n_win : ~0ull;
  wp.inv = 1.0 / (double)win_len;
  wp.inv_f = 1.0f / (float)win_len;

  KPA_CHECK(launch_fill_u32(w.counts, (u64)w.n_chunks * (RADIX + 1), 0, stream));
  KPA_CHECK(launch_fill_u32(w.counter, 1, 0, stream));
  KPA_CHECK(launch_fill_u32(w.status, w.n_tiles * RADIX, 0, stream));
  if (n) {
    // rows per workgroup: a power of two from BLOCK*PART_HIST_U up to
    // PART_HIST_ROWS (so that a chunk holds whole workgroups), small enough
    // that a bundle of a few hundred thousand rows still spreads over dozens
    // of workgroups
    u32 rpb = BLOCK * PART_HIST_U;
    while (rpb < PART_HIST_ROWS && (u64)rpb * 1024 < n) rpb <<= 1;
    KPA_LAUNCH("part_hist", k_part_hist, dim3((u32)ceil_div(n, rpb)), dim3(BLOCK), 0, stream, r,
               n, row_bytes, ts_off, ts_w, wp, w.counts, val_off, val_w, out_vals, rpb);
  }
  KPA_LAUNCH("part_scan", k_part_scan, dim3(1), dim3(BLOCK), 0, stream, w.counts, w.n_chunks,
             n_win, w.woff, out_win_off, out_oob);
  if (n) {
    const u32 grid = resident_grid(k_part_pass, (u32)w.n_tiles, PASS_THREADS);
    KPA_LAUNCH("part_pass", k_part_pass, dim3(grid), dim3(PASS_THREADS), 0, stream, r, n,
               row_bytes, key_off, ts_off, ts_w, wp, rid_base, rids_in, w.woff, (u32)w.n_tiles,
               w.status, w.counter, out_keys, out_rids);
  }
  return KPA_OK;
}

}  // namespace kpa

using namespace kpa;

extern "C" {

kpa_status kpa_partition_windows_workspace_size(uint64_t n, uint32_t n_win, size_t* bytes) {
  clear_error();
  KPA_REQUIRE(bytes != nullptr, KPA_EINVAL, "bytes is null");
  (void)n_win;
  Carver c(nullptr);
  PartWs w;
  part_plan(n, c, &w);
  *bytes = c.used + 256;
  return KPA_OK;
}

kpa_status kpa_partition_windows(const void* rows, uint64_t n, const kpa_row_layout* layout,
                                 uint64_t win_len, uint64_t win_origin, uint32_t n_win,
                                 uint32_t rid_base, uint64_t* out_keys, uint32_t* out_rids,
                                 uint64_t* out_vals, uint64_t* out_win_off, uint64_t* out_oob,
                                 void* ws, size_t ws_bytes, hipStream_t stream) {
  clear_error();
  KPA_CHECK(check_layout(layout, out_vals != nullptr, true));
  KPA_REQUIRE(!out_vals || aligned(out_vals, 8), KPA_EINVAL, "misaligned out_vals");
  KPA_REQUIRE(n_win >= 1 && n_win <= RADIX, KPA_EUNSUPPORTED, "n_win must be in [1, 256]");
  KPA_REQUIRE(win_len >= 1, KPA_EINVAL, "win_len must be >= 1");
  KPA_REQUIRE(out_win_off && out_oob && ws, KPA_EINVAL, "null pointer");
  KPA_REQUIRE(n < (1ull << 32) && n + rid_base <= (1ull << 32), KPA_EUNSUPPORTED,
              "n must be below 2^32 and rids must fit 32 bits");
  KPA_REQUIRE(n == 0 || (rows && out_keys && out_rids), KPA_EINVAL, "null pointer");
  KPA_REQUIRE(aligned(ws, 256) && aligned(out_win_off, 8) && aligned(out_oob, 8) &&
                  (n == 0 || (aligned(rows, 16) && aligned(out_keys, 8) && aligned(out_rids, 4))),
              KPA_EINVAL, "misaligned pointer");
  Carver c(ws);
  PartWs w;
  part_plan(n, c, &w);
  KPA_REQUIRE(c.used <= ws_bytes, KPA_EWORKSPACE, "workspace too small: need %zu bytes", c.used);
  return part_launch(static_cast<const unsigned char*>(rows), n, layout->row_bytes,
                     layout->key_off, layout->ts_off, layout->ts_w, layout->val_off,
                     layout->val_w, win_len, win_origin, n_win, rid_base, nullptr, out_keys,
                     out_rids, out_vals, out_win_off, out_oob, w, stream);
}

kpa_status kpa_partition_kpa(const uint64_t* keys, const uint32_t* rids, uint64_t n,
                             uint64_t win_len, uint64_t win_origin, uint32_t n_win,
                             uint64_t* out_keys, uint32_t* out_rids, uint64_t* out_win_off,
                             uint64_t* out_oob, void* ws, size_t ws_bytes, hipStream_t stream) {
  clear_error();
  KPA_REQUIRE(n_win >= 1 && n_win <= RADIX, KPA_EUNSUPPORTED, "n_win must be in [1, 256]");
  KPA_REQUIRE(win_len >= 1, KPA_EINVAL, "win_len must be >= 1");
  KPA_REQUIRE(out_win_off && out_oob && ws, KPA_EINVAL, "null pointer");
  KPA_REQUIRE(n < (1ull << 32), KPA_EUNSUPPORTED, "n must be below 2^32");
  KPA_REQUIRE(n == 0 || (keys && rids && out_keys && out_rids), KPA_EINVAL, "null pointer");
  KPA_REQUIRE(aligned(ws, 256) && aligned(out_win_off, 8) && aligned(out_oob, 8) &&
                  (n == 0 || (aligned(keys, 8) && aligned(rids, 4) && aligned(out_keys, 8) &&
                              aligned(out_rids, 4))),
              KPA_EINVAL, "misaligned pointer");
  Carver c(ws);
  PartWs w;
  part_plan(n, c, &w);
  KPA_REQUIRE(c.used <= ws_bytes, KPA_EWORKSPACE, "workspace too small: need %zu bytes", c.used);
  return part_launch(reinterpret_cast<const unsigned char*>(keys), n, 8, 0, 0, 8, 0, 8, win_len,
                     win_origin, n_win, 0, rids, out_keys, out_rids, nullptr, out_win_off,
                     out_oob, w, stream);
}

}  // extern "C"
