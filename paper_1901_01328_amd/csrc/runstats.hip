// Order statistics of the values inside each key run of a sorted KPA: the
// top-k values per key (Sec. 6 benchmark "TopK Per Key": the k largest values
// of every key in a window) and the number of distinct values per key (Sec. 6
// "Unique Count Per Key").  Both follow the paper's keyed aggregation: the
// KPA sorted on the key is scanned run by run and the nonresident value
// column is reached through the pointers (Table 2 keyed reduction).
//
// Runs come from the keyed reduction (key, count, first entry).  Work by run
// size:
//   c <= 16    one thread: values in registers, ranks by counting;
//   c <= 4096  one workgroup: values in LDS, bitonic sort;
//   larger     the run's values are gathered into a column in KPA order and
//              sorted in place by the onesweep radix passes (the big runs of
//              all segments form one device-counted segment list), then one
//              workgroup per run reads its sorted values.
#include "reduce_internal.hpp"
#include "sort_internal.hpp"

namespace kpa {

constexpr u32 RS_SMALL = 16;
constexpr u32 RS_MID = 4096;
constexpr u32 RS_TOPK_MAX = 16;
enum RsMode : u32 { RS_TOPK = 0, RS_UNIQUE = 1 };

struct RsSrc {
  const u32* rids;
  const unsigned char* rows;
  u32 row_bytes, val_off, val_w;
  __device__ __forceinline__ u64 val(u64 entry) const {
    return load_val(rows, rids[entry], row_bytes, val_off, val_w);
  }
};

struct RsOut {
  u64* topv;  // TOPK: run g's values at [gstart[g], gstart[g] + min(k, c)), descending
  u64* uniq;  // UNIQUE: distinct values of run g
  u32 k;
};

// Small runs in registers; larger runs are listed for the other kernels.
__global__ void __launch_bounds__(BLOCK) k_rs_small(RsSrc src, u32 mode, RsOut out,
                                                    const u64* __restrict__ gcnt,
                                                    const u64* __restrict__ gstart,
                                                    const u64* __restrict__ gseg_off, u32 n_seg,
                                                    u32* __restrict__ mid_list,
                                                    u32* __restrict__ big_list,
                                                    u32* __restrict__ counts) {
  const u64 G = gseg_off[n_seg];
  for (u64 g = (u64)blockIdx.x * BLOCK + threadIdx.x; g < G; g += (u64)gridDim.x * BLOCK) {
    const u64 c = gcnt[g], s = gstart[g];
    if (c > RS_SMALL) {
      if (c <= RS_MID) mid_list[atomicAdd(&counts[0], 1u)] = (u32)g;
      else big_list[atomicAdd(&counts[1], 1u)] = (u32)g;
      continue;
    }
    u64 v[RS_SMALL];
#pragma unroll
    for (u32 i = 0; i < RS_SMALL; ++i) v[i] = i < c ? src.val(s + i) : 0ull;
    if (mode == RS_UNIQUE) {
      u64 distinct = 0;
#pragma unroll
      for (u32 a = 0; a < RS_SMALL; ++a) {
        bool first = a < c;
#pragma unroll
        for (u32 b = 0; b < RS_SMALL; ++b) first = first && !(b < a && v[b] == v[a]);
        distinct += first;
      }
      out.uniq[g] = distinct;
    } else {
      // descending position of value a: larger values first, equal values
      // in entry order (the output is the multiset either way)
#pragma unroll
      for (u32 a = 0; a < RS_SMALL; ++a) {
        u32 r = 0;
#pragma unroll
        for (u32 b = 0; b < RS_SMALL; ++b)
          r += (b < c) & ((v[b] > v[a]) | ((v[b] == v[a]) & (b < a)));
        if (a < c && r < out.k) out.topv[s + r] = v[a];
      }
    }
  }
}

// Runs of up to 4096 entries: bitonic sort in LDS (ascending, padded with
// the largest value, so the run's values are the first c).
__global__ void __launch_bounds__(BLOCK) k_rs_mid(RsSrc src, u32 mode, RsOut out,
                                                  const u64* __restrict__ gcnt,
                                                  const u64* __restrict__ gstart,
                                                  const u32* __restrict__ list,
                                                  const u32* __restrict__ count) {
  __shared__ u64 v[RS_MID];
  __shared__ u32 red[WAVES];
  const u32 n = *count;
  for (u32 q = blockIdx.x; q < n; q += gridDim.x) {
    const u32 g = list[q];
    const u32 c = (u32)gcnt[g];
    const u64 s = gstart[g];
    u32 p2 = 1;
    while (p2 < c) p2 <<= 1;
    __syncthreads();
    for (u32 i = threadIdx.x; i < p2; i += BLOCK) v[i] = i < c ? src.val(s + i) : ~0ull;
    __syncthreads();
    for (u32 k = 2; k <= p2; k <<= 1) {
      for (u32 j = k >> 1; j > 0; j >>= 1) {
        for (u32 i = threadIdx.x; i < p2; i += BLOCK) {
          const u32 x = i ^ j;
          if (x > i) {
            const u64 a = v[i], b = v[x];
            if ((a > b) == ((i & k) == 0)) {
              v[i] = b;
              v[x] = a;
            }
          }
        }
        __syncthreads();
      }
    }
    if (mode == RS_UNIQUE) {
      u32 heads = 0;
      for (u32 i = threadIdx.x; i < c; i += BLOCK) heads += (i == 0 || v[i] != v[i - 1]);
      heads = wave_sum(heads);
      if (__lane_id() == 0) red[threadIdx.x >> 6] = heads;
      __syncthreads();
      if (threadIdx.x == 0) {
        u32 t = 0;
        for (int w = 0; w < WAVES; ++w) t += red[w];
        out.uniq[g] = t;
      }
    } else {
      const u32 t = min(out.k, c);
      if (threadIdx.x < t) out.topv[s + threadIdx.x] = v[c - 1 - threadIdx.x];
    }
  }
}

// Segment list of the big runs (their entry ranges in the KPA).
__global__ void __launch_bounds__(BLOCK) k_rs_big_list(const u64* __restrict__ gcnt,
                                                       const u64* __restrict__ gstart,
                                                       const u32* __restrict__ list,
                                                       const u32* __restrict__ count,
                                                       u64* __restrict__ lo,
                                                       u64* __restrict__ hi) {
  const u32 n = *count;
  for (u32 q = blockIdx.x * BLOCK + threadIdx.x; q < n; q += gridDim.x * BLOCK) {
    const u32 g = list[q];
    lo[q] = gstart[g];
    hi[q] = gstart[g] + gcnt[g];
  }
}

// Values of the big runs in KPA order, tile by tile (4096-entry tiles of the
// segment list).
__global__ void __launch_bounds__(BLOCK) k_rs_gather(RsSrc src, SegList sl,
                                                     const u32* __restrict__ tile_start,
                                                     const u32* __restrict__ tile_seg,
                                                     u64* __restrict__ vk) {
  const u32 n_seg = sl.n();
  const u32 total = tile_start[n_seg];
  for (u32 t = blockIdx.x; t < total; t += gridDim.x) {
    const u32 s = tile_seg[t];
    const u64 base = sl.lo[s] + (u64)(t - tile_start[s]) * TILE;
    const u64 end = min(sl.hi[s], base + TILE);
    for (u64 i = base + threadIdx.x; i < end; i += BLOCK) vk[i] = src.val(i);
  }
}

// One workgroup per big run, on its sorted values.
__global__ void __launch_bounds__(BLOCK) k_rs_big(u32 mode, RsOut out, const u64* __restrict__ vs,
                                                  const u64* __restrict__ gcnt,
                                                  const u64* __restrict__ gstart,
                                                  const u32* __restrict__ list,
                                                  const u32* __restrict__ count) {
  __shared__ u64 red[WAVES];
  const u32 n = *count;
  for (u32 q = blockIdx.x; q < n; q += gridDim.x) {
    const u32 g = list[q];
    const u64 c = gcnt[g], s = gstart[g];
    if (mode == RS_UNIQUE) {
      u64 heads = 0;
      for (u64 i = threadIdx.x; i < c; i += BLOCK) heads += (i == 0 || vs[s + i] != vs[s + i - 1]);
      heads = wave_sum(heads);
      __syncthreads();
      if (__lane_id() == 0) red[threadIdx.x >> 6] = heads;
      __syncthreads();
      if (threadIdx.x == 0) {
        u64 t = 0;
        for (int w = 0; w < WAVES; ++w) t += red[w];
        out.uniq[g] = t;
      }
    } else {
      const u32 t = (u32)min<u64>(out.k, c);
      if (threadIdx.x < t) out.topv[s + threadIdx.x] = vs[s + c - 1 - threadIdx.x];
    }
  }
}

struct RsWs {
  ReduceWs red;
  u64* gcnt;
  u64* gstart;
  u32* mid_list;
  u32* big_list;
  u32* counts;
  u64* big_lo;
  u64* big_hi;
  u64* vk;       // big runs' values in KPA order
  u64* vs;       // the same, sorted within each run
  u32* rid_out;  // payload output of the value sort (unused)
  u32* bt_start; // tiles of the big-run list
  u32* bt_seg;
  u64 big_max, bt_max;
  RadixWs rw;
};

static kpa_status rs_plan(u64 n_cap, u32 n_seg, Carver& c, RsWs* w) {
  reduce_plan(n_cap, n_seg, c, &w->red);
  const u64 cap = n_cap ? n_cap : 1;
  w->gcnt = c.take<u64>(cap);
  w->gstart = c.take<u64>(cap);
  w->mid_list = c.take<u32>(cap / (RS_SMALL + 1) + 1);
  w->big_max = cap / (RS_MID + 1) + 1;
  w->big_list = c.take<u32>(w->big_max);
  w->counts = c.take<u32>(2);
  w->big_lo = c.take<u64>(w->big_max);
  w->big_hi = c.take<u64>(w->big_max);
  w->vk = c.take<u64>(cap);
  w->vs = c.take<u64>(cap);
  w->rid_out = c.take<u32>(cap);
  w->bt_max = max_tiles(cap, (u32)w->big_max, TILE);
  w->bt_start = c.take<u32>(w->big_max + 1);
  w->bt_seg = c.take<u32>(w->bt_max);
  return radix_sort_plan(cap, (u32)w->big_max, c, &w->rw);
}

static kpa_status rs_launch(u32 mode, const u64* keys, const u32* rids, const u64* seg_off,
                            u32 n_seg, u64 n_cap, const unsigned char* rows,
                            const kpa_row_layout* L, u64* out_gkey, u64* out_gcnt,
                            u64* out_gstart, u64* out_gseg_off, RsOut o, const RsWs& w,
                            hipStream_t st) {
  u64* gcnt = out_gcnt ? out_gcnt : w.gcnt;
  u64* gstart = out_gstart ? out_gstart : w.gstart;
  ReduceOut ro{out_gkey, gcnt, nullptr, nullptr, gstart, out_gseg_off};
  KPA_CHECK(reduce_launch(keys, rids, seg_off, n_seg, nullptr, nullptr, false, ro, w.red, st));
  KPA_CHECK(launch_fill_u32(w.counts, 2, 0, st));
  RsSrc src{rids, rows, L->row_bytes, L->val_off, L->val_w};
  const u32 grid = (u32)std::min<u64>(ceil_div(n_cap ? n_cap : 1, BLOCK), 8192);
  KPA_LAUNCH("rs_small", k_rs_small, dim3(grid), dim3(BLOCK), 0, st, src, mode, o, gcnt, gstart,
             out_gseg_off, n_seg, w.mid_list, w.big_list, w.counts);
  KPA_LAUNCH("rs_mid", k_rs_mid, dim3(2048), dim3(BLOCK), 0, st, src, mode, o, gcnt, gstart,
             w.mid_list, w.counts);
  // big runs: gather their values, sort them in place per run, finish
  KPA_LAUNCH("rs_big_list", k_rs_big_list,
             dim3((u32)std::min<u64>(ceil_div(w.big_max, BLOCK), 1024)), dim3(BLOCK), 0, st,
             gcnt, gstart, w.big_list, w.counts + 1, w.big_lo, w.big_hi);
  const SegList sl{w.big_lo, w.big_hi, w.counts + 1, (u32)w.big_max};
  KPA_CHECK(launch_seg_tiles_list(sl, TILE, w.bt_start, st));
  KPA_CHECK(launch_tile_seg(w.bt_start, (u32)w.big_max, w.counts + 1, w.bt_max, w.bt_seg, st));
  KPA_LAUNCH("rs_gather", k_rs_gather, dim3((u32)std::min<u64>(w.bt_max, 8192)), dim3(BLOCK), 0, st,
             src, sl, w.bt_start, w.bt_seg, w.vk);
  KPA_CHECK(radix_sort_launch(w.vk, rids, w.vs, w.rid_out, sl, w.rw, st));
  KPA_LAUNCH("rs_big", k_rs_big, dim3(1024), dim3(BLOCK), 0, st, mode, o, w.vs, gcnt, gstart,
             w.big_list, w.counts + 1);
  return KPA_OK;
}

static kpa_status rs_check(const uint64_t* keys, const uint32_t* rids, const uint64_t* seg_off,
                           uint64_t n_cap, const void* rows, const kpa_row_layout* layout,
                           const uint64_t* out_gkey, const uint64_t* out_gseg_off, const void* ws) {
  KPA_CHECK(check_layout(layout, true, false));
  KPA_REQUIRE(keys && rids && seg_off && rows && out_gkey && out_gseg_off && ws, KPA_EINVAL,
              "null pointer");
  KPA_REQUIRE(aligned(keys, 8) && aligned(rids, 4) && aligned(seg_off, 8) && aligned(rows, 16) &&
                  aligned(out_gkey, 8) && aligned(out_gseg_off, 8) && aligned(ws, 256),
              KPA_EINVAL, "misaligned pointer");
  KPA_REQUIRE(n_cap < (1ull << 32), KPA_EUNSUPPORTED, "n_cap must be below 2^32");
  return KPA_OK;
}

}  // namespace kpa

using namespace kpa;

extern "C" {

kpa_status kpa_run_stats_workspace_size(uint64_t n_cap, uint32_t n_seg, size_t* bytes) {
  clear_error();
  KPA_REQUIRE(bytes, KPA_EINVAL, "bytes is null");
  Carver c(nullptr);
  RsWs w;
  KPA_CHECK(rs_plan(n_cap, n_seg ? n_seg : 1, c, &w));
  *bytes = c.used + 256;
  return KPA_OK;
}

kpa_status kpa_topk_per_key(const uint64_t* keys, const uint32_t* rids, const uint64_t* seg_off,
                            uint32_t n_seg, uint64_t n_cap, const void* rows,
                            const kpa_row_layout* layout, uint32_t k, uint64_t* out_gkey,
                            uint64_t* out_gcnt, uint64_t* out_gstart, uint64_t* out_topv,
                            uint64_t* out_gseg_off, void* ws, size_t ws_bytes,
                            hipStream_t stream) {
  clear_error();
  KPA_REQUIRE(k >= 1 && k <= RS_TOPK_MAX, KPA_EUNSUPPORTED, "k must be in [1, 16]");
  if (n_seg == 0) return KPA_OK;
  KPA_CHECK(rs_check(keys, rids, seg_off, n_cap, rows, layout, out_gkey, out_gseg_off, ws));
  KPA_REQUIRE(out_gcnt && out_gstart && out_topv, KPA_EINVAL, "null pointer");
  KPA_REQUIRE(aligned(out_gcnt, 8) && aligned(out_gstart, 8) && aligned(out_topv, 8), KPA_EINVAL,
              "misaligned pointer");
  Carver c(ws);
  RsWs w;
  KPA_CHECK(rs_plan(n_cap, n_seg, c, &w));
  KPA_REQUIRE(c.used <= ws_bytes, KPA_EWORKSPACE, "workspace too small: need %zu bytes", c.used);
  RsOut o{out_topv, nullptr, k};
  return rs_launch(RS_TOPK, keys, rids, seg_off, n_seg, n_cap,
                   static_cast<const unsigned char*>(rows), layout, out_gkey, out_gcnt,
                   out_gstart, out_gseg_off, o, w, stream);
}

kpa_status kpa_unique_count_by_key(const uint64_t* keys, const uint32_t* rids,
                                   const uint64_t* seg_off, uint32_t n_seg, uint64_t n_cap,
                                   const void* rows, const kpa_row_layout* layout,
                                   uint64_t* out_gkey, uint64_t* out_uniq, uint64_t* out_gseg_off,
                                   void* ws, size_t ws_bytes, hipStream_t stream) {
  clear_error();
  if (n_seg == 0) return KPA_OK;
  KPA_CHECK(rs_check(keys, rids, seg_off, n_cap, rows, layout, out_gkey, out_gseg_off, ws));
  KPA_REQUIRE(out_uniq && aligned(out_uniq, 8), KPA_EINVAL, "out_uniq null or misaligned");
  Carver c(ws);
  RsWs w;
  KPA_CHECK(rs_plan(n_cap, n_seg, c, &w));
  KPA_REQUIRE(c.used <= ws_bytes, KPA_EWORKSPACE, "workspace too small: need %zu bytes", c.used);
  RsOut o{nullptr, out_uniq, 0};
  return rs_launch(RS_UNIQUE, keys, rids, seg_off, n_seg, n_cap,
                   static_cast<const unsigned char*>(rows), layout, out_gkey, nullptr, nullptr,
                   out_gseg_off, o, w, stream);
}

}  // extern "C"
