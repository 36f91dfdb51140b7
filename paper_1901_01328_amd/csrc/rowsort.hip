// Grouping on full rows, without KPAs: the design the paper's ablation
// compares its KPAs with (Sec. 7.3, grouping that moves whole records).  The
// rows themselves are ordered by (window, key), stably, by nine onesweep
// passes over whole rows: the eight key bytes from least to most
// significant, then the window of the timestamp.  Every pass reads and
// writes each row whole (2 x row_bytes per row), where a KPA pass moves 12-
// byte entries.
//
// A pass ranks the tile's keys in LDS exactly as a KPA pass does (the
// payload is the row's index in the tile) and then copies each row from the
// tile's input (still in cache) to its destination, so that rows of one
// digit go out contiguously.
#include "digit_sort.hpp"

namespace kpa {

constexpr u32 ROW_PASSES = 9;  // 8 key bytes, then the window

struct RowSortParams {
  u32 row_words;  // 8-byte words per row: 2 or 4
  u32 key_word;   // the key's word in the row
  u32 ts_off, ts_w;
  u64 origin, win_len;
  u32 n_win;      // window digit of rows in no window
};

__device__ __forceinline__ u32 row_digit(const u64* __restrict__ rows, u64 e,
                                         const RowSortParams& p, u32 pass, u64 key) {
  if (pass < 8) return (u32)(key >> (8 * pass)) & 255u;
  const unsigned char* r = reinterpret_cast<const unsigned char*>(rows + e * p.row_words);
  const u64 ts = p.ts_w == 8 ? *reinterpret_cast<const u64*>(r + p.ts_off)
                             : (u64)*reinterpret_cast<const u32*>(r + p.ts_off);
  if (ts < p.origin) return p.n_win;
  const u64 q = (ts - p.origin) / p.win_len;
  return q < p.n_win ? (u32)q : p.n_win;
}

// The nine digit histograms of all rows (per-wave LDS counts, one global
// atomic per nonzero bin and workgroup).
__global__ void __launch_bounds__(BLOCK) k_rows_hist(const u64* __restrict__ rows, u64 n,
                                                     RowSortParams p, u32* __restrict__ hist) {
  __shared__ u32 h[WAVES][ROW_PASSES][RADIX];
  const u32 tid = threadIdx.x, w = tid >> 6;
  for (u32 i = tid; i < WAVES * ROW_PASSES * RADIX; i += BLOCK) (&h[0][0][0])[i] = 0;
  __syncthreads();
  for (u64 b = (u64)blockIdx.x * TILE; b < n; b += (u64)gridDim.x * TILE) {
#pragma unroll 4
    for (int j = 0; j < ITEMS; ++j) {
      const u64 e = b + tid + (u64)j * BLOCK;
      const bool v = e < n;
      const u64 key = v ? rows[e * p.row_words + p.key_word] : 0ull;
#pragma unroll
      for (u32 q = 0; q < ROW_PASSES; ++q)
        wave_hist_add(h[w][q], v ? row_digit(rows, e, p, q, key) : 0u, v);
    }
  }
  __syncthreads();
  for (u32 q = 0; q < ROW_PASSES; ++q) {
    u32 c = 0;
#pragma unroll
    for (int ww = 0; ww < WAVES; ++ww) c += h[ww][q][tid];
    if (c) atomicAdd(&hist[q * RADIX + tid], c);
  }
}

// Counts -> exclusive digit starts per pass (one workgroup per pass); the
// window pass also gives the caller its window offsets.
__global__ void __launch_bounds__(BLOCK) k_rows_scan(const u32* __restrict__ hist,
                                                     u32* __restrict__ base, u32 n_win,
                                                     u64* __restrict__ win_off,
                                                     u64* __restrict__ oob) {
  __shared__ u32 sc[WAVES + 1];
  const u32 q = blockIdx.x, tid = threadIdx.x;
  const u32 c = hist[q * RADIX + tid];
  u32 tot;
  const u32 ex = block_excl_sum(c, sc, &tot);
  base[q * RADIX + tid] = ex;
  if (q == ROW_PASSES - 1) {
    if (tid <= n_win) win_off[tid] = ex;
    if (tid == n_win) *oob = c;
  }
}

// One pass: persistent workgroups claim tiles in order; the look-back chain
// runs over the whole array (one segment, fewer than 2^30 rows).
template <int RW>
__global__ void __launch_bounds__(PASS_THREADS, PASS_WAVES / 2)
    k_rows_pass(const u64* __restrict__ in, u64* __restrict__ out, u64 n, RowSortParams p,
                u32 pass, const u32* __restrict__ base, u32 n_tiles, u32* __restrict__ status,
                u32* __restrict__ counter) {
  __shared__ OnesweepSmemT<PASS_WAVES> sm;
  const u32 tid = threadIdx.x;
  const u64 my_base = tid < RADIX ? (u64)base[pass * RADIX + tid] : 0ull;
  while (true) {
    __syncthreads();
    if (tid == 0) sm.tile = atomicAdd(counter, 1u);
    __syncthreads();
    const u32 t = sm.tile;
    if (t >= n_tiles) return;
    const u64 t0 = (u64)t * TILE;
    u64 kk[PASS_ITEMS];
    u32 rr[PASS_ITEMS], dd[PASS_ITEMS];
    u32 valid = 0;
#pragma unroll
    for (int j = 0; j < PASS_ITEMS; ++j) {
      const u32 o = tile_offset_t<PASS_WAVES>(j);
      const u64 e = t0 + o;
      kk[j] = e < n ? in[e * RW + p.key_word] : 0ull;
      rr[j] = o;
      dd[j] = e < n ? row_digit(in, e, p, pass, kk[j]) : 0u;
      if (e < n) valid |= 1u << j;
    }
    u32 tile_count;
    const u32 cnt_d = onesweep_rank_stage(sm, kk, rr, dd, valid, status, t, t, &tile_count);
    onesweep_lookback(sm, status, t, t, cnt_d, tile_count, my_base);
    // rows out: staged entry i goes to gbase[d] + (i - lstart[d])
    for (u32 i = tid; i < sm.count; i += PASS_THREADS) {
      const u32 d = sm.sdig[i];
      const u64 dst = sm.gbase[d] + (i - sm.lstart[d]);
      const uint4* s = reinterpret_cast<const uint4*>(in + (t0 + sm.srids[i]) * RW);
      uint4* o = reinterpret_cast<uint4*>(out + dst * RW);
#pragma unroll
      for (int w = 0; w < RW / 2; ++w) o[w] = s[w];
    }
  }
}

struct RowSortWs {
  u64* tmp;
  u32* hist;
  u32* base;
  u32* status;
  u32* counter;
  u64 n_tiles;
};

static void rowsort_plan(u64 n, u32 row_bytes, Carver& c, RowSortWs* w) {
  w->n_tiles = ceil_div(n ? n : 1, TILE);
  w->tmp = c.take<u64>((n ? n : 1) * (row_bytes / 8));
  w->hist = c.take<u32>(ROW_PASSES * RADIX);
  w->base = c.take<u32>(ROW_PASSES * RADIX);
  w->status = c.take<u32>(w->n_tiles * RADIX);
  w->counter = c.take<u32>(1);
}

}  // namespace kpa

using namespace kpa;

extern "C" {

kpa_status kpa_sort_rows_windowed_workspace_size(uint64_t n, uint32_t row_bytes, size_t* bytes) {
  clear_error();
  KPA_REQUIRE(bytes, KPA_EINVAL, "bytes is null");
  KPA_REQUIRE(row_bytes == 16 || row_bytes == 32, KPA_EUNSUPPORTED, "row_bytes must be 16 or 32");
  Carver c(nullptr);
  RowSortWs w;
  rowsort_plan(n, row_bytes, c, &w);
  *bytes = c.used + 256;
  return KPA_OK;
}

kpa_status kpa_sort_rows_windowed(const void* rows, uint64_t n, const kpa_row_layout* layout,
                                  uint64_t win_len, uint64_t win_origin, uint32_t n_win,
                                  void* out_rows, uint64_t* out_win_off, uint64_t* out_oob,
                                  void* ws, size_t ws_bytes, hipStream_t stream) {
  clear_error();
  KPA_CHECK(check_layout(layout, false, true));
  KPA_REQUIRE(layout->row_bytes == 16 || layout->row_bytes == 32, KPA_EUNSUPPORTED,
              "row_bytes must be 16 or 32");
  KPA_REQUIRE(n_win >= 1 && n_win < RADIX, KPA_EUNSUPPORTED, "n_win must be in [1, 255]");
  KPA_REQUIRE(win_len >= 1, KPA_EINVAL, "win_len must be >= 1");
  KPA_REQUIRE(n < MAX_SEG_ENTRIES, KPA_EUNSUPPORTED, "n must be below 2^30");
  KPA_REQUIRE(out_win_off && out_oob && ws && (n == 0 || (rows && out_rows)), KPA_EINVAL,
              "null pointer");
  KPA_REQUIRE(rows != out_rows || n == 0, KPA_EINVAL, "rows must not alias out_rows");
  KPA_REQUIRE(aligned(ws, 256) && aligned(out_win_off, 8) && aligned(out_oob, 8) &&
                  (n == 0 || (aligned(rows, 16) && aligned(out_rows, 16))),
              KPA_EINVAL, "misaligned pointer");
  Carver c(ws);
  RowSortWs w;
  rowsort_plan(n, layout->row_bytes, c, &w);
  KPA_REQUIRE(c.used <= ws_bytes, KPA_EWORKSPACE, "workspace too small: need %zu bytes", c.used);
  RowSortParams p;
  p.row_words = layout->row_bytes / 8;
  p.key_word = layout->key_off / 8;
  p.ts_off = layout->ts_off;
  p.ts_w = layout->ts_w;
  p.origin = win_origin;
  p.win_len = win_len;
  p.n_win = n_win;
  const u64* in = static_cast<const u64*>(rows);
  u64* out = static_cast<u64*>(out_rows);
  KPA_CHECK(launch_fill_u32(w.hist, ROW_PASSES * RADIX, 0, stream));
  if (n) {
    KPA_LAUNCH("rows_hist", k_rows_hist, dim3((u32)std::min<u64>(w.n_tiles, 4096)), dim3(BLOCK),
               0, stream, in, n, p, w.hist);
  }
  KPA_LAUNCH("rows_scan", k_rows_scan, dim3(ROW_PASSES), dim3(BLOCK), 0, stream, w.hist, w.base,
             n_win, out_win_off, out_oob);
  if (!n) return KPA_OK;
  for (u32 pass = 0; pass < ROW_PASSES; ++pass) {
    // pass p writes out for even p and the workspace copy for odd p, so the
    // ninth pass (p = 8) lands in out_rows
    const u64* src = pass == 0 ? in : ((pass - 1) % 2 == 0 ? out : w.tmp);
    u64* dst = pass % 2 == 0 ? out : w.tmp;
    KPA_CHECK(launch_fill_u32(w.status, w.n_tiles * RADIX, 0, stream));
    KPA_CHECK(launch_fill_u32(w.counter, 1, 0, stream));
    if (p.row_words == 4) {
      const u32 grid = resident_grid(k_rows_pass<4>, (u32)w.n_tiles, PASS_THREADS);
      KPA_LAUNCH("rows_pass", k_rows_pass<4>, dim3(grid), dim3(PASS_THREADS), 0, stream, src, dst,
                 n, p, pass, w.base, (u32)w.n_tiles, w.status, w.counter);
    } else {
      const u32 grid = resident_grid(k_rows_pass<2>, (u32)w.n_tiles, PASS_THREADS);
      KPA_LAUNCH("rows_pass", k_rows_pass<2>, dim3(grid), dim3(PASS_THREADS), 0, stream, src, dst,
                 n, p, pass, w.base, (u32)w.n_tiles, w.status, w.counter);
    }
  }
  return KPA_OK;
}

}  // extern "C"
