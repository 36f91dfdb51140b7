// Learned-splitter sort: model evaluation, workspace layout, launch entry.
#pragma once

#include "sort_internal.hpp"

namespace kpa {

constexpr u32 FCAP = TILE;        // entries sorted on chip by one workgroup
constexpr u32 FH = FCAP / 2;      // chunk stride of the finishing pass
constexpr u32 BUCKET_TARGET = 1024;  // mean bucket size the bucket count aims at
constexpr u32 MAX_BUCKET_BITS = 16;

// Per-segment model state prepared on the device from a kpa_pwl_model.
struct SegModel {
  u64 kmin, kmax;
  float scale;         // n_seg / (kmax - kmin), 0 when kmax == kmin
  u32 nseg;            // PWL segments
  u32 bits;            // log2 of the bucket count (0: one bucket)
  u32 valid;           // knots checked: finite, within [0,1], nondecreasing
  const float* knots;  // n_seg + 1 values
};

// F(key): 0..1, nondecreasing in key for nondecreasing knots.  key <= kmin maps
// to knots[0], key >= kmax to 1; between, linear interpolation clamped to the
// segment's two knots.  Each step (u64->float conversion, product with a
// positive scale, truncation, fraction, a + f*(b-a) with b >= a, clamp) is
// monotone under round-to-nearest, and segment j's values lie in
// [knots[j], knots[j+1]], so F never decreases.  Written without branches so
// that the knot loads of many keys can be in flight together.
__device__ __forceinline__ float pwl_eval(const SegModel& m, u64 key) {
  const u64 span = m.kmax - m.kmin;
  u64 d = key > m.kmin ? key - m.kmin : 0ull;
  d = d < span ? d : span;
  const float x = (float)d * m.scale;
  u32 j = (u32)x;
  j = j >= m.nseg ? m.nseg - 1 : j;
  const float f = x - (float)j;
  const float a = m.knots[j], b = m.knots[j + 1];
  float F = a + f * (b - a);
  F = F < a ? a : F;
  F = F > b ? b : F;
  F = key <= m.kmin ? m.knots[0] : F;
  return key >= m.kmax ? 1.0f : F;
}

__device__ __forceinline__ u32 model_bucket(const SegModel& m, u64 key) {
  if (m.bits == 0) return 0u;
  const float B = (float)(1u << m.bits);
  const u32 b = (u32)(pwl_eval(m, key) * B);
  const u32 top = (1u << m.bits) - 1;
  return b > top ? top : b;
}

// Bucket id refined by 8 more bits: floor(F * 2^(bits+8)), capped.  Scaling
// by a power of two is exact, so model_fine(k) >> 8 == model_bucket(k) for
// every key (bits <= 16, so the product stays below 2^24 and exact).
__device__ __forceinline__ u32 model_fine(const SegModel& m, u64 key) {
  const float B = (float)(1u << (m.bits + 8));
  const u32 b = (u32)(pwl_eval(m, key) * B);
  const u32 top = (1u << (m.bits + 8)) - 1;
  return b > top ? top : b;
}

struct LearnedWs {
  u64* keys_tmp;   // scatter ping-pong buffer; later the fallback's input
  u32* rids_tmp;
  SegModel* segm;  // n_seg
  u64* cur_min;    // n_seg: smallest and largest key of each segment
  u64* cur_max;
  u32* ltile_start;  // tile map of the scatter passes (n_seg + 1)
  u32* ftile_start;  // tile map of the finishing pass (n_seg + 1)
  u32* ltile_seg;    // segment of each scatter tile (max_tiles)
  u32* ftile_seg;    // segment of each finishing stretch (max_ftiles)
  u32* hist;       // n_seg * 8 * 256 (only 2 passes used)
  u32* seg_mask;
  u32* status0;
  u32* status1;
  u32* counters;
  OrderBufs order;
  u64* fb_lo;      // oversize chunks: [lo, hi)
  u64* fb_hi;
  u64* fb_rhi;     // hi for chunks to re-sort, lo for single-key chunks
  u64* fb_min;
  u64* fb_max;
  u32* fb_count;
  u32* fb_tile_start;
  u32* fb_tile_seg;  // segment of each tile of the chunk lists
  // pivot rounds: the oversize chunks of round r are split three ways around
  // their most frequent key; parts still larger than FCAP go to round r+1
  u64* rl_lo[2];
  u64* rl_hi[2];
  u32* rl_count;     // [2] round lists, [2] small-range list
  u64* sm_lo;        // parts of at most FCAP entries, sorted on chip
  u64* sm_hi;
  u64* pivot;
  u64* cnt3;         // per chunk: below, equal, above the pivot
  u32* p_hist;       // digit offsets for the pivot scatter (n * 8 * 256)
  u32* p_mask;
  u32* p_tile_start;
  u64 n_cap;
  u64 max_tiles;
  u64 max_ftiles;
  u32 max_fb;
  RadixWs fb_radix;  // radix sort of the re-sorted chunks
};

kpa_status learned_sort_plan(u64 n_cap, u32 n_seg, Carver& c, LearnedWs* w);
kpa_status learned_sort_launch(const u64* keys_in, const u32* rids_in, u64* keys_out,
                               u32* rids_out, const SegList& sl, const kpa_pwl_model* models,
                               kpa_sort_stats* stats, const LearnedWs& lw, hipStream_t st);

}  // namespace kpa
