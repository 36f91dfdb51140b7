// Learned-splitter sort: model evaluation, workspace layout, launch entry.
#pragma once

#include "sort_internal.hpp"

namespace kpa {

constexpr u32 FCAP = TILE;        // entries sorted on chip by one workgroup
constexpr u32 FH = FCAP / 2;      // chunk stride of the finishing pass
constexpr u32 BUCKET_LOG2 = 9;  // default mean bucket size the bucket count aims at: 2^9
#ifndef KPA_REFINE_BITS
#define KPA_REFINE_BITS 8
#endif
constexpr u32 REFINE_BITS = KPA_REFINE_BITS;  // bits of F below the bucket id used by the finish
constexpr u32 MAX_BUCKET_BITS = 16;

// Per-segment model state prepared on the device from a kpa_pwl_model.
struct SegModel {
  u64 kmin, kmax;      // the segment's own key range (from a sample of its keys)
  float scale;         // nseg / hspan, 0 when hspan == 0
  u32 nseg;            // PWL segments
  u32 bits;            // log2 of the bucket count (0: one bucket)
  u32 valid;           // knots checked: finite, within [0, 1], nondecreasing
  u32 sh;              // key - kmin is shifted right by sh to fit 32 bits
  u32 hspan;           // (kmax - kmin) >> sh
  const float* knots;  // nseg + 1 values in global memory (copied to LDS for use)
};

// The knots are read from LDS through a pointer of the LDS address space, so
// that each evaluation is one two-word LDS read.
typedef __attribute__((address_space(3))) const float lds_float;
typedef __attribute__((address_space(1))) const float global_float;

// All threads of the workgroup: copy the segment's knots to `lds` (at least
// nseg + 1 floats; nseg <= KPA_PWL_MAX_SEG for every prepared model).  The
// caller synchronizes before the first evaluation.
__device__ __forceinline__ const lds_float* bind_knots(const SegModel& m, float* lds) {
  const global_float* g = (const global_float*)m.knots;
  for (u32 j = threadIdx.x; j <= m.nseg; j += blockDim.x) lds[j] = g[j];
  return (const lds_float*)lds;
}

// F(key): 0..1, nondecreasing in key for nondecreasing knots.  The offset
// key - kmin (0 for keys below kmin), shifted right by sh (so that it fits 32
// bits) and capped at hspan (keys above kmax), is converted to float and
// scaled to the segment axis: x = h*scale in [0, nseg].  F interpolates the
// two knots of segment j = floor(x) (capped at nseg - 1) at the fraction
// f = h*scale - j (one fused rounding) and is clamped to them.  Each step is
// monotone under round-to-nearest and segment j's values lie in
// [knots[j], knots[j+1]], so F never decreases.  The two fused operations
// are written out so that every kernel evaluating the model computes the
// same bits, whatever the compiler would contract.
template <class KP>
__device__ __forceinline__ float pwl_eval(const SegModel& m, const KP* kn, u64 key) {
  const u64 d = key > m.kmin ? (key - m.kmin) >> m.sh : 0ull;
  // the capped offset fits 32 bits: clamp on the two halves and convert from
  // u32 (the same value, so the same float, as converting the u64)
  const u32 dlo = (u32)d;
  const u32 h = (u32)(d >> 32) != 0u ? m.hspan : (dlo < m.hspan ? dlo : m.hspan);
  const float hf = __uint2float_rn(h);
  const float x = hf * m.scale;
  u32 j = (u32)x;
  j = j < m.nseg - 1 ? j : m.nseg - 1;
  const float f = fmaf(hf, m.scale, -(float)j);
  const float a = kn[j], b = kn[j + 1];
  return __builtin_amdgcn_fmed3f(fmaf(f, b - a, a), a, b);
}

// With bits == 0 the cap is 0, so every key is in bucket 0 without a branch
// (a branch per key would keep the compiler from overlapping the knot reads
// of a thread's keys).
template <class KP>
__device__ __forceinline__ u32 model_bucket(const SegModel& m, const KP* kn, u64 key) {
  const float B = (float)(1u << m.bits);
  const u32 b = (u32)(pwl_eval(m, kn, key) * B);
  const u32 top = (1u << m.bits) - 1;
  return b > top ? top : b;
}

// Bucket id refined by REFINE_BITS more bits: floor(F * 2^(bits+REFINE_BITS)),
// capped.  Scaling by a power of two is exact, so model_fine(k) >> REFINE_BITS
// == model_bucket(k) for every key.
template <class KP>
__device__ __forceinline__ u32 model_fine(const SegModel& m, const KP* kn, u64 key) {
  const float B = (float)(1u << (m.bits + REFINE_BITS));
  const u32 b = (u32)(pwl_eval(m, kn, key) * B);
  const u32 top = (1u << (m.bits + REFINE_BITS)) - 1;
  return b > top ? top : b;
}

struct LearnedWs {
  u64* keys_tmp;   // scatter ping-pong buffer; later the fallback's input
  u32* rids_tmp;
  u64* vals_tmp;   // the same for a value column (planned with one only, else null)
  SegModel* segm;  // n_seg
  u64* cur_min;    // n_seg: smallest and largest sampled key of each segment
  u64* cur_max;
  u32* ltile_start;  // tile map of the scatter passes (n_seg + 1)
  u32* ftile_start;  // tile map of the finishing pass (n_seg + 1)
  u32* ltile_seg;    // segment of each scatter tile (max_tiles)
  u32* ftile_seg;    // segment of each finishing stretch (max_ftiles)
  u64* factive;      // stretches that hold a bucket start: segment << 32 | index (max_ftiles)
  u32* fedge;        // per stretch: offset of its first bucket start, NONE if none (max_ftiles)
  u32* fn_active;
  u32* hist;       // n_seg * 8 * 256 (only 2 passes used)
  u32* seg_mask;
  u32* status0;
  u32* status1;
  u32* counters;
  OrderBufs order;
  u64* fb_lo;      // oversize chunks: [lo, hi)
  u64* fb_hi;
  u32* fb_seg;     // segment of each oversize chunk (its model sorts the chunk's small parts)
  u64* fb_min;
  u64* fb_max;
  u32* fb_count;
  u32* fb_tile_start;
  u32* fb_tile_seg;  // segment of each tile of the chunk lists
  // pivot rounds: the oversize chunks of round r are split three ways around
  // their most frequent key; parts still larger than FCAP go to round r+1
  u64* rl_lo[2];
  u64* rl_hi[2];
  u32* rl_seg[2];
  u32* rl_count;     // [2] round lists, [2] small-range list
  u64* sm_lo;        // parts of at most FCAP entries, sorted on chip
  u64* sm_hi;
  u32* sm_seg;
  u64* pivot;
  u64* cnt3;         // per chunk: below, equal, above the pivot
  u32* p_mask;       // per chunk: 1 when it is split (holds more than its pivot key)
  u32* t_lt;         // per tile of the chunk list: entries below / equal to the pivot,
  u32* t_eq;         // then their counts in the chunk's earlier tiles
  uint16_t* t_eqbits;  // per tile and thread: which of the thread's 16 entries equal the pivot
  u64 n_cap;
  u64 max_tiles;
  u64 max_ftiles;
  u32 max_fb;
  RadixWs fb_radix;  // radix sort of the re-sorted chunks
};

// vals: also plan for a value column.
kpa_status learned_sort_plan(u64 n_cap, u32 n_seg, Carver& c, LearnedWs* w, bool vals = false);
// vals_in/vals_out (both or neither; the plan must have had vals): a value
// column that follows the keys' permutation.
// bucket_log2: the mean bucket size the bucket count aims at is 2^bucket_log2.
kpa_status learned_sort_launch(const u64* keys_in, const u32* rids_in, u64* keys_out,
                               u32* rids_out, const SegList& sl, const kpa_pwl_model* models,
                               kpa_sort_stats* stats, const LearnedWs& lw, hipStream_t st,
                               const u64* vals_in = nullptr, u64* vals_out = nullptr,
                               u32 bucket_log2 = BUCKET_LOG2);

}  // namespace kpa
