// Select (Table 2: keep the (key, pointer) pairs that pass a predicate, in
// their order; ParDo filters run as Select over a KPA, Sec. 4.2), the unkeyed
// reduction over windows (Table 2 "Unkeyed reduction"; Sec. 6 "Windowed
// Average All"), and the pane concatenation that builds sliding windows out
// of slide-length partitions (Sec. 4.2 "Windowing": the slide length is the
// range of each partition of a sliding window).
//
// Select predicate per segment s: x * den[s] <op> num[s], with x the resident
// key or the value reached through the pointer, the product exact in 128 bits
// and num[s] a 128-bit integer, so a threshold that is a ratio (such as an
// average sum/count) is compared without rounding.
//
// Select runs over 4096-entry tiles: count the survivors per tile, an
// exclusive scan of the counts (the outputs of all segments are back to back),
// then write each tile's survivors in order.
#include "reduce_internal.hpp"

namespace kpa {

constexpr u32 RADIX_WIN = 256;  // most windows of an unkeyed window reduction

struct SelPred {
  const u64* num_lo;
  const u64* num_hi;  // may be null (0)
  const u64* den;     // may be null (1)
  const unsigned char* rows;
  u32 row_bytes, val_off, val_w;
  u32 column;  // 0 key, 1 value
  u32 op;      // kpa_select_op
  __device__ __forceinline__ bool pass(u64 key, u32 rid, u32 seg) const {
    const u64 x = column == 0 ? key : load_val(rows, rid, row_bytes, val_off, val_w);
    const u64 d = den ? den[seg] : 1ull;
    const u64 lo = x * d, hi = __umul64hi(x, d);
    const u64 nlo = num_lo[seg], nhi = num_hi ? num_hi[seg] : 0ull;
    const bool gt = hi > nhi || (hi == nhi && lo > nlo);
    const bool eq = hi == nhi && lo == nlo;
    switch (op) {
      case KPA_SEL_GT: return gt;
      case KPA_SEL_GE: return gt || eq;
      case KPA_SEL_LT: return !gt && !eq;
      case KPA_SEL_LE: return !gt;
      case KPA_SEL_EQ: return eq;
      default: return !eq;
    }
  }
};

struct SelTile {
  u32 seg;
  u64 base;
  u32 cnt;
};

__device__ __forceinline__ SelTile sel_tile(const u64* seg_off, const u32* tile_start,
                                            const u32* tile_seg, u32 tile) {
  SelTile r;
  r.seg = tile_seg[tile];
  const u64 a = seg_off[r.seg], b = seg_off[r.seg + 1];
  r.base = a + (u64)(tile - tile_start[r.seg]) * TILE;
  r.cnt = r.base < b ? (u32)min<u64>(TILE, b - r.base) : 0u;
  return r;
}

// Thread t tests entries t*ITEMS .. t*ITEMS+ITEMS-1 of the tile (staged
// through LDS so that the loads are coalesced) and returns its pass bits.
__device__ __forceinline__ u32 sel_flags(const u64* keys, const u32* rids, const SelTile& tr,
                                         const SelPred& pr, u64* sk, u32* sr, u64 (&k)[ITEMS],
                                         u32 (&r)[ITEMS]) {
  const u32 tid = threadIdx.x;
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const u32 i = tid + j * BLOCK;
    k[j] = i < tr.cnt ? keys[tr.base + i] : 0ull;
    r[j] = i < tr.cnt ? rids[tr.base + i] : 0u;
  }
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const u32 i = tid + j * BLOCK;
    sk[i + (i >> 4)] = k[j];
    sr[i + (i >> 4)] = r[j];
  }
  __syncthreads();
  u32 bits = 0;
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const u32 i = tid * ITEMS + j;
    k[j] = sk[i + (i >> 4)];
    r[j] = sr[i + (i >> 4)];
    if (i < tr.cnt && pr.pass(k[j], r[j], tr.seg)) bits |= 1u << j;
  }
  return bits;
}

constexpr u32 SEL_PT = TILE + TILE / 16;

__global__ void __launch_bounds__(BLOCK) k_sel_count(const u64* __restrict__ keys,
                                                     const u32* __restrict__ rids,
                                                     const u64* __restrict__ seg_off,
                                                     const u32* __restrict__ tile_start,
                                                     const u32* __restrict__ tile_seg, u32 n_seg,
                                                     SelPred pr, u32* __restrict__ tcount) {
  __shared__ u64 sk[SEL_PT];
  __shared__ u32 sr[SEL_PT];
  __shared__ u32 red[WAVES];
  const u32 tile = blockIdx.x;
  if (tile >= tile_start[n_seg]) return;
  const SelTile tr = sel_tile(seg_off, tile_start, tile_seg, tile);
  u64 k[ITEMS];
  u32 r[ITEMS];
  const u32 bits = sel_flags(keys, rids, tr, pr, sk, sr, k, r);
  const u32 c = wave_sum((u32)__popc(bits));
  if (__lane_id() == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    u32 t = 0;
    for (int w = 0; w < WAVES; ++w) t += red[w];
    tcount[tile] = t;
  }
}

__global__ void __launch_bounds__(BLOCK) k_sel_write(const u64* __restrict__ keys,
                                                     const u32* __restrict__ rids,
                                                     const u64* __restrict__ seg_off,
                                                     const u32* __restrict__ tile_start,
                                                     const u32* __restrict__ tile_seg, u32 n_seg,
                                                     SelPred pr, const u64* __restrict__ tbase,
                                                     u64* __restrict__ out_keys,
                                                     u32* __restrict__ out_rids) {
  __shared__ u64 sk[SEL_PT];
  __shared__ u32 sr[SEL_PT];
  __shared__ u32 sc[WAVES + 1];
  const u32 tile = blockIdx.x;
  if (tile >= tile_start[n_seg]) return;
  const SelTile tr = sel_tile(seg_off, tile_start, tile_seg, tile);
  u64 k[ITEMS];
  u32 r[ITEMS];
  const u32 bits = sel_flags(keys, rids, tr, pr, sk, sr, k, r);
  u32 tot;
  const u32 ex = block_excl_sum((u32)__popc(bits), sc, &tot);
  u64 o = tbase[tile] + ex;
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    if ((bits >> j) & 1u) {
      out_keys[o] = k[j];
      out_rids[o] = r[j];
      ++o;
    }
  }
}

struct SelWs {
  u32* tile_start;
  u32* tile_seg;
  u32* tcount;
  u64* tbase;
  u64* bsum;
  u64 max_tiles;
};

static void sel_plan(u64 n_cap, u32 n_seg, Carver& c, SelWs* w) {
  w->max_tiles = max_tiles(n_cap, n_seg, TILE);
  w->tile_start = c.take<u32>((u64)n_seg + 1);
  w->tile_seg = c.take<u32>(w->max_tiles);
  w->tcount = c.take<u32>(w->max_tiles);
  w->tbase = c.take<u64>(w->max_tiles);
  w->bsum = c.take<u64>(ceil_div(w->max_tiles, SCAN_TILES));
}

// ---------------------------------------------------------------- unkeyed --
// Per window: count, the value sum split into the sums of the values' low
// and high 32-bit halves (each below n * 2^32 < 2^64, so exact), and the
// maximum.  The 128-bit total is assembled at the end.

struct RallAcc {
  u64 cnt, lo, hi, mx;
};

constexpr u32 RALL_ROWS = 1u << 16;  // rows per workgroup
constexpr int RALL_U = 8;            // row loads in flight per thread

__device__ __forceinline__ bool rall_window(u64 ts, u64 origin, u64 win_len, u32 n_win, u32& w) {
  if (ts < origin) return false;
  const u64 q = (ts - origin) / win_len;
  if (q >= n_win) return false;
  w = (u32)q;
  return true;
}

__global__ void __launch_bounds__(BLOCK) k_rall(const unsigned char* __restrict__ rows, u64 n,
                                                u32 row_bytes, u32 val_off, u32 val_w, u32 ts_off,
                                                u32 ts_w, u64 origin, u64 win_len, u32 n_win,
                                                RallAcc* __restrict__ acc) {
  __shared__ u64 s_cnt[RADIX_WIN + 1], s_lo[RADIX_WIN + 1], s_hi[RADIX_WIN + 1],
      s_mx[RADIX_WIN + 1];
  const u32 tid = threadIdx.x;
  for (u32 i = tid; i <= RADIX_WIN; i += BLOCK) s_cnt[i] = s_lo[i] = s_hi[i] = s_mx[i] = 0;
  __syncthreads();
  const u64 r0 = (u64)blockIdx.x * RALL_ROWS, r1 = min(n, r0 + RALL_ROWS);
  // running accumulation of this thread's current window, flushed on change
  u32 cw = 0xFFFFFFFFu;
  u64 c = 0, lo = 0, hi = 0, mx = 0;
  auto flush = [&]() {
    if (cw != 0xFFFFFFFFu && c) {
      atomicAdd(reinterpret_cast<unsigned long long*>(&s_cnt[cw]), c);
      atomicAdd(reinterpret_cast<unsigned long long*>(&s_lo[cw]), lo);
      atomicAdd(reinterpret_cast<unsigned long long*>(&s_hi[cw]), hi);
      atomicMax(reinterpret_cast<unsigned long long*>(&s_mx[cw]), mx);
    }
    c = lo = hi = mx = 0;
  };
  for (u64 b = r0; b < r1; b += (u64)BLOCK * RALL_U) {
    u64 ts[RALL_U], vv[RALL_U];
#pragma unroll
    for (int j = 0; j < RALL_U; ++j) {
      const u64 i = b + tid + (u64)j * BLOCK;
      ts[j] = vv[j] = 0;
      if (i < r1) {
        const unsigned char* row = rows + i * row_bytes;
        ts[j] = ts_w == 8 ? *reinterpret_cast<const u64*>(row + ts_off)
                          : (u64)*reinterpret_cast<const u32*>(row + ts_off);
        vv[j] = val_w == 8 ? *reinterpret_cast<const u64*>(row + val_off)
                           : (u64)*reinterpret_cast<const u32*>(row + val_off);
      }
    }
#pragma unroll
    for (int j = 0; j < RALL_U; ++j) {
      const u64 i = b + tid + (u64)j * BLOCK;
      u32 w;
      if (i < r1 && rall_window(ts[j], origin, win_len, n_win, w)) {
        if (w != cw) {
          flush();
          cw = w;
        }
        c += 1;
        lo += vv[j] & 0xFFFFFFFFull;
        hi += vv[j] >> 32;
        mx = vv[j] > mx ? vv[j] : mx;
      } else if (i < r1) {
        atomicAdd(reinterpret_cast<unsigned long long*>(&s_cnt[RADIX_WIN]), 1ull);
      }
    }
  }
  flush();
  __syncthreads();
  for (u32 w = tid; w < n_win; w += BLOCK) {
    if (s_cnt[w]) {
      atomicAdd(reinterpret_cast<unsigned long long*>(&acc[w].cnt), s_cnt[w]);
      atomicAdd(reinterpret_cast<unsigned long long*>(&acc[w].lo), s_lo[w]);
      atomicAdd(reinterpret_cast<unsigned long long*>(&acc[w].hi), s_hi[w]);
      atomicMax(reinterpret_cast<unsigned long long*>(&acc[w].mx), s_mx[w]);
    }
  }
  if (tid == 0 && s_cnt[RADIX_WIN])
    atomicAdd(reinterpret_cast<unsigned long long*>(&acc[RADIX_WIN].cnt), s_cnt[RADIX_WIN]);
}

__global__ void __launch_bounds__(BLOCK) k_rall_final(const RallAcc* __restrict__ acc, u32 n_win,
                                                      u64* __restrict__ out_cnt,
                                                      u64* __restrict__ out_lo,
                                                      u64* __restrict__ out_hi,
                                                      u64* __restrict__ out_max,
                                                      u64* __restrict__ out_oob) {
  for (u32 w = threadIdx.x; w < n_win; w += BLOCK) {
    const RallAcc a = acc[w];
    // sum = hi * 2^32 + lo, as a 128-bit integer
    const u64 s_lo = (a.hi << 32) + a.lo;
    const u64 carry = s_lo < a.lo ? 1ull : 0ull;
    if (out_cnt) out_cnt[w] = a.cnt;
    if (out_lo) out_lo[w] = s_lo;
    if (out_hi) out_hi[w] = (a.hi >> 32) + carry;
    if (out_max) out_max[w] = a.mx;
  }
  if (threadIdx.x == 0 && out_oob) *out_oob = acc[RADIX_WIN].cnt;
}

// -------------------------------------------------------- sliding windows --
// Window w of a sliding window over panes (slide-length partitions) covers
// panes w .. w+P-1; its entries are the concatenation of those panes' groups,
// as (key, group index) pairs.

__global__ void __launch_bounds__(1024) k_panes_off(const u64* __restrict__ gseg_off, u32 n_win,
                                                    u32 P, u64* __restrict__ out_seg_off) {
  __shared__ u64 wsum[16];
  const u32 tid = threadIdx.x, lane = __lane_id(), wv = tid >> 6;
  u64 carry = 0;
  for (u32 w0 = 0; w0 < n_win; w0 += 1024) {
    const u32 w = w0 + tid;
    const u64 len = w < n_win ? gseg_off[w + P] - gseg_off[w] : 0ull;
    u64 incl = len;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const u64 t = __shfl_up(incl, o, 64);
      if (lane >= (u32)o) incl += t;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    u64 pre = carry;
    for (u32 i = 0; i < wv; ++i) pre += wsum[i];
    if (w < n_win) out_seg_off[w] = pre + incl - len;
    u64 tot = 0;
    for (int i = 0; i < 16; ++i) tot += wsum[i];
    __syncthreads();
    carry += tot;
  }
  if (tid == 0) out_seg_off[n_win] = carry;
}

__global__ void __launch_bounds__(BLOCK) k_panes_fill(const u64* __restrict__ gkey,
                                                      const u64* __restrict__ gseg_off, u32 n_win,
                                                      u32 P, const u64* __restrict__ out_seg_off,
                                                      u64 cap, u64* __restrict__ out_keys,
                                                      u32* __restrict__ out_rids) {
  // grid.y = window; grid.x strides over its entries
  const u32 w = blockIdx.y;
  if (w >= n_win) return;
  const u64 g0 = gseg_off[w], len = gseg_off[w + P] - g0, o0 = out_seg_off[w];
  for (u64 j = (u64)blockIdx.x * BLOCK + threadIdx.x; j < len; j += (u64)gridDim.x * BLOCK) {
    if (o0 + j < cap) {
      out_keys[o0 + j] = gkey[g0 + j];
      out_rids[o0 + j] = (u32)(g0 + j);
    }
  }
}

}  // namespace kpa

using namespace kpa;

extern "C" {

kpa_status kpa_select_workspace_size(uint64_t n_cap, uint32_t n_seg, size_t* bytes) {
  clear_error();
  KPA_REQUIRE(bytes, KPA_EINVAL, "bytes is null");
  Carver c(nullptr);
  SelWs w;
  sel_plan(n_cap, n_seg ? n_seg : 1, c, &w);
  *bytes = c.used + 256;
  return KPA_OK;
}

kpa_status kpa_select(const uint64_t* keys, const uint32_t* rids, const uint64_t* seg_off,
                      uint32_t n_seg, uint64_t n_cap, const void* rows,
                      const kpa_row_layout* layout, kpa_select_column column, kpa_select_op op,
                      const uint64_t* num_lo, const uint64_t* num_hi, const uint64_t* den,
                      uint64_t* out_keys, uint32_t* out_rids, uint64_t* out_seg_off, void* ws,
                      size_t ws_bytes, hipStream_t stream) {
  clear_error();
  KPA_REQUIRE(column == KPA_SEL_KEY || column == KPA_SEL_VALUE, KPA_EINVAL, "bad column");
  KPA_REQUIRE(op >= KPA_SEL_GT && op <= KPA_SEL_NE, KPA_EINVAL, "bad op");
  if (column == KPA_SEL_VALUE) KPA_CHECK(check_layout(layout, true, false));
  if (n_seg == 0) return KPA_OK;
  KPA_REQUIRE(keys && rids && seg_off && num_lo && out_keys && out_rids && out_seg_off && ws,
              KPA_EINVAL, "null pointer");
  KPA_REQUIRE(column == KPA_SEL_KEY || rows, KPA_EINVAL, "rows needed to test the value");
  KPA_REQUIRE(aligned(keys, 8) && aligned(rids, 4) && aligned(seg_off, 8) && aligned(num_lo, 8) &&
                  aligned(num_hi, 8) && aligned(den, 8) && aligned(out_keys, 8) &&
                  aligned(out_rids, 4) && aligned(out_seg_off, 8) && aligned(ws, 256) &&
                  (!rows || aligned(rows, 16)),
              KPA_EINVAL, "misaligned pointer");
  KPA_REQUIRE(n_cap < (1ull << 32), KPA_EUNSUPPORTED, "n_cap must be below 2^32");
  Carver c(ws);
  SelWs w;
  sel_plan(n_cap, n_seg, c, &w);
  KPA_REQUIRE(c.used <= ws_bytes, KPA_EWORKSPACE, "workspace too small: need %zu bytes", c.used);
  SelPred pr;
  pr.num_lo = num_lo;
  pr.num_hi = num_hi;
  pr.den = den;
  pr.rows = static_cast<const unsigned char*>(rows);
  pr.row_bytes = layout ? layout->row_bytes : 8;
  pr.val_off = layout ? layout->val_off : 0;
  pr.val_w = layout ? layout->val_w : 8;
  pr.column = (u32)column;
  pr.op = (u32)op;
  KPA_CHECK(launch_seg_tiles(seg_off, nullptr, n_seg, TILE, w.tile_start, stream));
  KPA_CHECK(launch_tile_seg(w.tile_start, n_seg, nullptr, w.max_tiles, w.tile_seg, stream));
  KPA_LAUNCH("select_count", k_sel_count, dim3((u32)w.max_tiles), dim3(BLOCK), 0, stream, keys,
             rids, seg_off, w.tile_start, w.tile_seg, n_seg, pr, w.tcount);
  KPA_CHECK(launch_tile_scan(w.tcount, w.tile_start, w.tile_seg, n_seg, w.max_tiles, w.bsum,
                             w.tbase, out_seg_off, stream));
  KPA_LAUNCH("select_write", k_sel_write, dim3((u32)w.max_tiles), dim3(BLOCK), 0, stream, keys,
             rids, seg_off, w.tile_start, w.tile_seg, n_seg, pr, w.tbase, out_keys, out_rids);
  return KPA_OK;
}

kpa_status kpa_reduce_all_windows_workspace_size(uint32_t n_win, size_t* bytes) {
  clear_error();
  KPA_REQUIRE(bytes, KPA_EINVAL, "bytes is null");
  (void)n_win;
  *bytes = sizeof(RallAcc) * (RADIX_WIN + 1) + 256;
  return KPA_OK;
}

kpa_status kpa_reduce_all_windows(const void* rows, uint64_t n, const kpa_row_layout* layout,
                                  uint64_t win_len, uint64_t win_origin, uint32_t n_win,
                                  uint64_t* out_cnt, uint64_t* out_sum_lo, uint64_t* out_sum_hi,
                                  uint64_t* out_max, uint64_t* out_oob, void* ws, size_t ws_bytes,
                                  hipStream_t stream) {
  clear_error();
  KPA_CHECK(check_layout(layout, true, true));
  KPA_REQUIRE(n_win >= 1 && n_win <= RADIX_WIN, KPA_EUNSUPPORTED, "n_win must be in [1, 256]");
  KPA_REQUIRE(win_len >= 1, KPA_EINVAL, "win_len must be >= 1");
  KPA_REQUIRE(ws && (n == 0 || rows), KPA_EINVAL, "null pointer");
  KPA_REQUIRE(n < (1ull << 32), KPA_EUNSUPPORTED, "n must be below 2^32");
  KPA_REQUIRE(aligned(ws, 256) && (n == 0 || aligned(rows, 16)) && aligned(out_cnt, 8) &&
                  aligned(out_sum_lo, 8) && aligned(out_sum_hi, 8) && aligned(out_max, 8) &&
                  aligned(out_oob, 8),
              KPA_EINVAL, "misaligned pointer");
  KPA_REQUIRE(ws_bytes >= sizeof(RallAcc) * (RADIX_WIN + 1), KPA_EWORKSPACE,
              "workspace too small: need %zu bytes", sizeof(RallAcc) * (RADIX_WIN + 1));
  RallAcc* acc = static_cast<RallAcc*>(ws);
  KPA_CHECK(launch_fill_u64(reinterpret_cast<u64*>(acc), 4ull * (RADIX_WIN + 1), 0, stream));
  if (n) {
    KPA_LAUNCH("reduce_all", k_rall, dim3((u32)ceil_div(n, RALL_ROWS)), dim3(BLOCK), 0, stream,
               static_cast<const unsigned char*>(rows), n, layout->row_bytes, layout->val_off,
               layout->val_w, layout->ts_off, layout->ts_w, win_origin, win_len, n_win, acc);
  }
  KPA_LAUNCH("reduce_all_final", k_rall_final, dim3(1), dim3(BLOCK), 0, stream, acc, n_win,
             out_cnt, out_sum_lo, out_sum_hi, out_max, out_oob);
  return KPA_OK;
}

kpa_status kpa_window_panes(const uint64_t* gkey, const uint64_t* gseg_off, uint32_t n_pane,
                            uint32_t panes_per_window, uint64_t* out_keys, uint32_t* out_rids,
                            uint64_t* out_seg_off, uint64_t out_cap, hipStream_t stream) {
  clear_error();
  KPA_REQUIRE(panes_per_window >= 1 && panes_per_window <= n_pane, KPA_EINVAL,
              "panes_per_window must be in [1, n_pane]");
  KPA_REQUIRE(gkey && gseg_off && out_keys && out_rids && out_seg_off, KPA_EINVAL,
              "null pointer");
  KPA_REQUIRE(aligned(gkey, 8) && aligned(gseg_off, 8) && aligned(out_keys, 8) &&
                  aligned(out_rids, 4) && aligned(out_seg_off, 8),
              KPA_EINVAL, "misaligned pointer");
  const u32 n_win = n_pane - panes_per_window + 1;
  KPA_REQUIRE(n_win <= 65535, KPA_EUNSUPPORTED, "at most 65535 windows");
  KPA_LAUNCH("panes_off", k_panes_off, dim3(1), dim3(1024), 0, stream, gseg_off, n_win,
             panes_per_window, out_seg_off);
  KPA_LAUNCH("panes_fill", k_panes_fill, dim3(256, n_win), dim3(BLOCK), 0, stream, gkey, gseg_off,
             n_win, panes_per_window, out_seg_off, out_cap, out_keys, out_rids);
  return KPA_OK;
}

}  // extern "C"
