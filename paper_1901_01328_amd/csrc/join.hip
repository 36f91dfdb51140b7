// Join (Table 2: two sorted KPAs, one sequential pass; Sec. 4.2 "Temporal
// Join": two records of the same window and key form a pair).
//
// Both sorted KPAs are first reduced to their runs of equal keys (count, sum
// of values, first entry), per window.  A pair of runs with the same key
// contributes count_L * count_R pairs and sum_L * sum_R to the sum of value
// products (the integers mod 2^64 form a ring, so the product of the sums is
// the sum of the products).  The two run lists are intersected by merge path
// over their combined length, split into 4096-entry tiles per window: in
// merge order a run of L sits immediately before the R run with the same key
// (keys are unique within each list, ties go to L), so a matching R run lies
// in the same tile or is the first R run of the next tile.  Pairs, when asked
// for, are written per matching key as the L entries (in KPA order) times the
// R entries, keys ascending, windows in order.
#include "reduce_internal.hpp"

namespace kpa {

constexpr u32 JT = TILE;  // merged run-list entries per tile

__device__ __forceinline__ u64 list_split(const u64* a, u64 na, const u64* b, u64 nb, u64 d) {
  u64 lo = d > nb ? d - nb : 0, hi = d < na ? d : na;
  while (lo < hi) {
    const u64 mid = (lo + hi) >> 1;
    if (a[mid] <= b[d - mid - 1]) lo = mid + 1; else hi = mid;
  }
  return lo;
}

struct JoinSides {
  const u64 *gk_l, *gc_l, *gs_l, *gst_l, *goff_l;
  const u64 *gk_r, *gc_r, *gs_r, *gst_r, *goff_r;
};

__global__ void __launch_bounds__(BLOCK) k_join_splits(JoinSides js, const u32* __restrict__ tile_start,
                                                       u32 n_seg, u64* __restrict__ split,
                                                       u32 max_t) {
  const u32 total = min(tile_start[n_seg], max_t);  // split holds max_t entries
  for (u32 t = blockIdx.x * BLOCK + threadIdx.x; t < total; t += gridDim.x * BLOCK) {
    const u32 s = find_seg(tile_start, n_seg, t);
    const u64 l0 = js.goff_l[s], nl = js.goff_l[s + 1] - l0;
    const u64 r0 = js.goff_r[s], nr = js.goff_r[s + 1] - r0;
    const u64 d = min((u64)(t - tile_start[s]) * JT, nl + nr);
    split[t] = list_split(js.gk_l + l0, nl, js.gk_r + r0, nr, d);
  }
}

struct JoinSmem {
  u64 rk[JT];
  u64 red[2 * WAVES];
  u64 scan[WAVES + 1];
};

// EMIT = false: per-window count and sum of products, per-tile pair totals.
// EMIT = true: pairs written at tile offsets (exclusive scan of the totals).
template <bool EMIT>
__global__ void __launch_bounds__(BLOCK) k_join_match(JoinSides js, const u32* __restrict__ tile_start,
                                                      u32 n_seg, const u64* __restrict__ split,
                                                      u64* __restrict__ out_count,
                                                      u64* __restrict__ out_sumprod,
                                                      u64* __restrict__ tile_pairs,
                                                      const u32* __restrict__ rids_l,
                                                      const u32* __restrict__ rids_r,
                                                      u64* __restrict__ pairs, u64 pairs_cap) {
  __shared__ JoinSmem sm;
  const u32 tile = blockIdx.x;
  if (tile >= tile_start[n_seg]) return;
  const u32 s = find_seg(tile_start, n_seg, tile);
  const u32 t_in = tile - tile_start[s];
  const u64 l0 = js.goff_l[s], nl = js.goff_l[s + 1] - l0;
  const u64 r0 = js.goff_r[s], nr = js.goff_r[s + 1] - r0;
  const u64 d0 = (u64)t_in * JT, d1 = min(d0 + JT, nl + nr);
  if (d0 >= d1) {
    if (!EMIT && threadIdx.x == 0) tile_pairs[tile] = 0;
    return;
  }
  const bool last = tile + 1 >= tile_start[s + 1];
  const u64 i0 = split[tile], i1 = last ? nl : split[tile + 1];
  const u64 j0 = d0 - i0, j1 = d1 - i1;
  const u32 la = (u32)(i1 - i0), lb = (u32)(j1 - j0);
  for (u32 x = threadIdx.x; x < lb; x += BLOCK) sm.rk[x] = js.gk_r[r0 + j0 + x];
  __syncthreads();
  // when pairs are emitted, thread t takes L runs [t*16, t*16+16) of the
  // tile, in order (its pairs then follow those of thread t-1)
  u64 cnt = 0, sp = 0, npairs = 0;
  const u32 a0 = threadIdx.x * ITEMS, a1 = min(la, a0 + ITEMS);
  // R run matching L run a of the tile, or ~0
  auto match = [&](u32 a) -> u64 {
    const u64 key = js.gk_l[l0 + i0 + a];
    u32 lo = 0, hi = lb;
    while (lo < hi) {
      const u32 mid = (lo + hi) >> 1;
      if (sm.rk[mid] < key) lo = mid + 1; else hi = mid;
    }
    if (lo < lb && sm.rk[lo] == key) return j0 + lo;
    if (a + 1 == la && j1 < nr && js.gk_r[r0 + j1] == key) return j1;
    return ~0ull;
  };
  if (!EMIT) {
    // Totals only: the order of the runs does not matter, so lane i of a wave
    // takes run i of each 256-run stretch and the loads of the L runs (and of
    // the matched R runs, which ascend with them) coalesce.
    for (u32 a = threadIdx.x; a < la; a += BLOCK) {
      const u64 jm = match(a);
      if (jm != ~0ull) {
        const u64 cl = js.gc_l[l0 + i0 + a], cr = js.gc_r[r0 + jm];
        cnt += cl * cr;
        sp += js.gs_l[l0 + i0 + a] * js.gs_r[r0 + jm];
      }
    }
    cnt = wave_sum(cnt);
    sp = wave_sum(sp);
    __syncthreads();
    if (__lane_id() == 0) {
      sm.red[threadIdx.x >> 6] = cnt;
      sm.red[WAVES + (threadIdx.x >> 6)] = sp;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      u64 c = 0, p = 0;
      for (int i = 0; i < WAVES; ++i) {
        c += sm.red[i];
        p += sm.red[WAVES + i];
      }
      if (c) atomicAdd(reinterpret_cast<unsigned long long*>(out_count + s), (unsigned long long)c);
      if (p) atomicAdd(reinterpret_cast<unsigned long long*>(out_sumprod + s), (unsigned long long)p);
      tile_pairs[tile] = c;
    }
    return;
  }
  for (u32 a = a0; a < a1; ++a) {
    const u64 jm = match(a);
    if (jm != ~0ull) npairs += js.gc_l[l0 + i0 + a] * js.gc_r[r0 + jm];
  }
  // exclusive scan of the threads' pair counts (u64) within the tile
  u64 incl = npairs;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const u64 t = __shfl_up(incl, o, 64);
    if (__lane_id() >= (u32)o) incl += t;
  }
  if (__lane_id() == 63) sm.scan[threadIdx.x >> 6] = incl;
  __syncthreads();
  u64 off = tile_pairs[tile] + incl - npairs;  // tile_pairs holds exclusive tile offsets
  for (u32 w = 0; w < (threadIdx.x >> 6); ++w) off += sm.scan[w];
  for (u32 a = a0; a < a1; ++a) {
    const u64 jm = match(a);
    if (jm == ~0ull) continue;
    const u64 li = l0 + i0 + a, ri = r0 + jm;
    const u64 key = js.gk_l[li];
    const u64 cl = js.gc_l[li], cr = js.gc_r[ri];
    const u64 sl = js.gst_l[li], sr = js.gst_r[ri];
    for (u64 x = 0; x < cl; ++x) {
      const u64 rl = rids_l[sl + x];
      for (u64 y = 0; y < cr; ++y) {
        const u64 o = off + x * cr + y;
        if (o < pairs_cap) {
          pairs[3 * o + 0] = key;
          pairs[3 * o + 1] = rl;
          pairs[3 * o + 2] = rids_r[sr + y];
        }
      }
    }
    off += cl * cr;
  }
}

// One workgroup: exclusive scan of per-tile pair totals, and the grand total.
__global__ void __launch_bounds__(1024) k_join_scan(u64* __restrict__ tile_pairs,
                                                    const u32* __restrict__ tile_start, u32 n_seg,
                                                    u64* __restrict__ total_out) {
  __shared__ u64 wh[17];
  const u32 n = tile_start[n_seg];
  const u32 per = (n + 1023) / 1024;
  const u32 t0 = min(n, threadIdx.x * per), t1 = min(n, t0 + per);
  u64 h = 0;
  for (u32 t = t0; t < t1; ++t) h += tile_pairs[t];
  u64 inc = h;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const u64 x = __shfl_up(inc, o, 64);
    if (__lane_id() >= (u32)o) inc += x;
  }
  if (__lane_id() == 63) wh[threadIdx.x >> 6] = inc;
  __syncthreads();
  u64 run = inc - h;
  for (u32 w = 0; w < (threadIdx.x >> 6); ++w) run += wh[w];
  for (u32 t = t0; t < t1; ++t) {
    const u64 c = tile_pairs[t];
    tile_pairs[t] = run;
    run += c;
  }
  if (threadIdx.x == 1023) wh[16] = run;
  __syncthreads();
  if (threadIdx.x == 0 && total_out) *total_out = wh[16];
}

struct JoinWs {
  ReduceWs red;
  u64 *gk_l, *gc_l, *gs_l, *gst_l, *goff_l;
  u64 *gk_r, *gc_r, *gs_r, *gst_r, *goff_r;
  u32* tile_start;
  u64* split;
  u64* tile_pairs;
  u64 max_tiles;
};

static void join_plan(u64 nl, u64 nr, u32 n_seg, Carver& c, JoinWs* w) {
  reduce_plan(nl > nr ? nl : nr, n_seg, c, &w->red);
  const u64 L = nl ? nl : 1, R = nr ? nr : 1;
  w->gk_l = c.take<u64>(L);
  w->gc_l = c.take<u64>(L);
  w->gs_l = c.take<u64>(L);
  w->gst_l = c.take<u64>(L);
  w->goff_l = c.take<u64>((u64)n_seg + 1);
  w->gk_r = c.take<u64>(R);
  w->gc_r = c.take<u64>(R);
  w->gs_r = c.take<u64>(R);
  w->gst_r = c.take<u64>(R);
  w->goff_r = c.take<u64>((u64)n_seg + 1);
  w->max_tiles = max_tiles(nl + nr, n_seg, JT);
  w->tile_start = c.take<u32>((u64)n_seg + 1);
  w->split = c.take<u64>(w->max_tiles);
  w->tile_pairs = c.take<u64>(w->max_tiles);
}

// Workspace of a join over run lists given by the caller: the merge-path
// tiles only.
struct JoinRunsWs {
  u32* tile_start;
  u64* split;
  u64* tile_pairs;
  u64 max_tiles;
};

static void join_runs_plan(u64 gl, u64 gr, u32 n_seg, Carver& c, JoinRunsWs* w) {
  w->max_tiles = max_tiles(gl + gr, n_seg, JT);
  w->tile_start = c.take<u32>((u64)n_seg + 1);
  w->split = c.take<u64>(w->max_tiles);
  w->tile_pairs = c.take<u64>(w->max_tiles);
}

}  // namespace kpa

using namespace kpa;

extern "C" {

kpa_status kpa_join_workspace_size(uint64_t nl_cap, uint64_t nr_cap, uint32_t n_seg,
                                   size_t* bytes) {
  clear_error();
  KPA_REQUIRE(bytes, KPA_EINVAL, "bytes is null");
  Carver c(nullptr);
  JoinWs w;
  join_plan(nl_cap, nr_cap, n_seg ? n_seg : 1, c, &w);
  *bytes = c.used + 256;
  return KPA_OK;
}

kpa_status kpa_join(const uint64_t* lk, const uint32_t* lr, const uint64_t* l_seg_off,
                    uint64_t nl_cap, const uint64_t* rk, const uint32_t* rr,
                    const uint64_t* r_seg_off, uint64_t nr_cap, uint32_t n_seg,
                    const void* rows_l, const void* rows_r, const kpa_row_layout* layout,
                    uint64_t* out_count, uint64_t* out_sumprod, uint64_t* out_pairs,
                    uint64_t pairs_cap, uint64_t* out_npairs, void* ws, size_t ws_bytes,
                    hipStream_t stream) {
  clear_error();
  KPA_CHECK(check_layout(layout, true, false));
  if (n_seg == 0) return KPA_OK;
  KPA_REQUIRE(l_seg_off && r_seg_off && out_count && out_sumprod && ws, KPA_EINVAL, "null pointer");
  KPA_REQUIRE((nl_cap == 0 || (lk && lr && rows_l)) && (nr_cap == 0 || (rk && rr && rows_r)),
              KPA_EINVAL, "null pointer");
  KPA_REQUIRE(aligned(ws, 256) && aligned(out_count, 8) && aligned(out_sumprod, 8) &&
                  (!out_pairs || aligned(out_pairs, 8)) && (!out_npairs || aligned(out_npairs, 8)),
              KPA_EINVAL, "misaligned pointer");
  KPA_REQUIRE(nl_cap < (1ull << 32) && nr_cap < (1ull << 32), KPA_EUNSUPPORTED,
              "inputs must hold fewer than 2^32 entries");
  Carver c(ws);
  JoinWs w;
  join_plan(nl_cap, nr_cap, n_seg, c, &w);
  KPA_REQUIRE(c.used <= ws_bytes, KPA_EWORKSPACE, "workspace too small: need %zu bytes", c.used);

  // runs of each side: key, count, sum of values, first entry
  ReduceOut ol{w.gk_l, w.gc_l, w.gs_l, nullptr, w.gst_l, w.goff_l};
  if (nl_cap) {
    KPA_CHECK(reduce_launch(lk, lr, l_seg_off, n_seg, static_cast<const unsigned char*>(rows_l),
                            layout, true, ol, w.red, stream));
  } else {
    KPA_CHECK(launch_fill_u64(w.goff_l, (u64)n_seg + 1, 0, stream));
  }
  ReduceOut orr{w.gk_r, w.gc_r, w.gs_r, nullptr, w.gst_r, w.goff_r};
  if (nr_cap) {
    KPA_CHECK(reduce_launch(rk, rr, r_seg_off, n_seg, static_cast<const unsigned char*>(rows_r),
                            layout, true, orr, w.red, stream));
  } else {
    KPA_CHECK(launch_fill_u64(w.goff_r, (u64)n_seg + 1, 0, stream));
  }
  KPA_CHECK(launch_fill_u64(out_count, n_seg, 0, stream));
  KPA_CHECK(launch_fill_u64(out_sumprod, n_seg, 0, stream));
  JoinSides js{w.gk_l, w.gc_l, w.gs_l, w.gst_l, w.goff_l, w.gk_r, w.gc_r, w.gs_r, w.gst_r, w.goff_r};
  KPA_CHECK(launch_seg_tiles(w.goff_l, w.goff_r, n_seg, JT, w.tile_start, stream));
  KPA_LAUNCH("join_splits", k_join_splits, dim3((u32)std::min<u64>(ceil_div(w.max_tiles, BLOCK), 4096)),
             dim3(BLOCK), 0, stream, js, w.tile_start, n_seg, w.split, (u32)w.max_tiles);
  KPA_LAUNCH("join_match", k_join_match<false>, dim3((u32)w.max_tiles), dim3(BLOCK), 0, stream, js,
             w.tile_start, n_seg, w.split, out_count, out_sumprod, w.tile_pairs, lr, rr, out_pairs,
             pairs_cap);
  if (out_pairs || out_npairs) {
    KPA_LAUNCH("join_scan", k_join_scan, dim3(1), dim3(1024), 0, stream, w.tile_pairs, w.tile_start,
               n_seg, out_npairs);
  }
  if (out_pairs && pairs_cap) {
    KPA_LAUNCH("join_emit", k_join_match<true>, dim3((u32)w.max_tiles), dim3(BLOCK), 0, stream, js,
               w.tile_start, n_seg, w.split, out_count, out_sumprod, w.tile_pairs, lr, rr,
               out_pairs, pairs_cap);
  }
  return KPA_OK;
}

kpa_status kpa_join_runs_workspace_size(uint64_t gl_cap, uint64_t gr_cap, uint32_t n_seg,
                                        size_t* bytes) {
  clear_error();
  KPA_REQUIRE(bytes, KPA_EINVAL, "bytes is null");
  Carver c(nullptr);
  JoinRunsWs w;
  join_runs_plan(gl_cap, gr_cap, n_seg ? n_seg : 1, c, &w);
  *bytes = c.used + 256;
  return KPA_OK;
}

kpa_status kpa_join_runs(const uint64_t* l_gkey, const uint64_t* l_cnt, const uint64_t* l_sum,
                         const uint64_t* l_gseg_off, uint64_t gl_cap, const uint64_t* r_gkey,
                         const uint64_t* r_cnt, const uint64_t* r_sum, const uint64_t* r_gseg_off,
                         uint64_t gr_cap, uint32_t n_seg, uint64_t* out_count,
                         uint64_t* out_sumprod, void* ws, size_t ws_bytes, hipStream_t stream) {
  clear_error();
  if (n_seg == 0) return KPA_OK;
  KPA_REQUIRE(l_gseg_off && r_gseg_off && out_count && out_sumprod && ws, KPA_EINVAL,
              "null pointer");
  KPA_REQUIRE((gl_cap == 0 || (l_gkey && l_cnt && l_sum)) &&
                  (gr_cap == 0 || (r_gkey && r_cnt && r_sum)),
              KPA_EINVAL, "null pointer");
  KPA_REQUIRE(aligned(l_gkey, 8) && aligned(l_cnt, 8) && aligned(l_sum, 8) &&
                  aligned(r_gkey, 8) && aligned(r_cnt, 8) && aligned(r_sum, 8) &&
                  aligned(l_gseg_off, 8) && aligned(r_gseg_off, 8) && aligned(out_count, 8) &&
                  aligned(out_sumprod, 8) && aligned(ws, 256),
              KPA_EINVAL, "misaligned pointer");
  KPA_REQUIRE(gl_cap < (1ull << 32) && gr_cap < (1ull << 32), KPA_EUNSUPPORTED,
              "run lists must hold fewer than 2^32 groups");
  Carver c(ws);
  JoinRunsWs w;
  join_runs_plan(gl_cap, gr_cap, n_seg, c, &w);
  KPA_REQUIRE(c.used <= ws_bytes, KPA_EWORKSPACE, "workspace too small: need %zu bytes", c.used);
  KPA_CHECK(launch_fill_u64(out_count, n_seg, 0, stream));
  KPA_CHECK(launch_fill_u64(out_sumprod, n_seg, 0, stream));
  // group starts are needed only to emit pairs, which this call does not
  JoinSides js{l_gkey, l_cnt, l_sum, nullptr, l_gseg_off, r_gkey, r_cnt, r_sum, nullptr,
               r_gseg_off};
  KPA_CHECK(launch_seg_tiles(l_gseg_off, r_gseg_off, n_seg, JT, w.tile_start, stream));
  KPA_LAUNCH("join_splits", k_join_splits, dim3((u32)std::min<u64>(ceil_div(w.max_tiles, BLOCK), 4096)),
             dim3(BLOCK), 0, stream, js, w.tile_start, n_seg, w.split, (u32)w.max_tiles);
  KPA_LAUNCH("join_match", k_join_match<false>, dim3((u32)w.max_tiles), dim3(BLOCK), 0, stream, js,
             w.tile_start, n_seg, w.split, out_count, out_sumprod, w.tile_pairs, nullptr, nullptr,
             nullptr, 0);
  return KPA_OK;
}

}  // extern "C"
