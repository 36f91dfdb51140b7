// Sort (Table 2: KPA(c) -> KPA(c), sequential access) as a segmented
// least-significant-digit radix sort with 8-bit digits.
//
// Launch sequence (all segments together, sizes read from device memory):
//   1. tile map: tile_start[s] for 4096-entry tiles of each segment;
//   2. one histogram pass counting all eight digits of every key per segment;
//   3. per segment: exclusive digit offsets, and a mask of the passes whose
//      digit is not constant over the segment (constant digits need no pass);
//   4. eight onesweep scatter passes; a segment only takes part in its active
//      passes and ping-pongs between the output and a workspace buffer so that
//      its last active pass lands in the output (a segment with no active pass
//      is copied).
// Each scatter is stable, so the sort is stable: ties keep input order.
//
// The histogram and scatter kernels are templates over the digit function
// (digit_sort.hpp) so that the learned-splitter sort reuses them with model
// buckets as digits.
#include "digit_sort.hpp"

namespace kpa {

struct RadixDF {
  static constexpr int PASSES = 8;
  static constexpr int SMEM = 1;
  __device__ __forceinline__ void bind(float*) {}
  struct Params {};
  struct Staged {};
  RadixDF() = default;
  __device__ __forceinline__ RadixDF(const Params&, u32) {}
  __device__ __forceinline__ explicit RadixDF(const Staged&) {}
  static __device__ __forceinline__ Staged fetch(const Params&, u32) { return Staged{}; }
  __device__ __forceinline__ void bind_staged(const Staged&, float*) {}
  __device__ __forceinline__ u32 digit(u64 k, u32 pass) const {
    return (u32)(k >> (8 * pass)) & 255u;
  }
  __device__ __forceinline__ void digits(u64 k, u32 (&d)[PASSES]) const {
#pragma unroll
    for (int p = 0; p < PASSES; ++p) d[p] = (u32)(k >> (8 * p)) & 255u;
  }
};

__global__ void __launch_bounds__(1024) k_seg_tiles_list(SegList sl, u32 tile,
                                                         u32* __restrict__ tile_start) {
  __shared__ u32 sm[17];
  const u32 n_seg = sl.n();
  const u32 per = (n_seg + 1023) / 1024;
  const u32 s0 = min(n_seg, threadIdx.x * per);
  const u32 s1 = min(n_seg, s0 + per);
  u32 local = 0;
  for (u32 s = s0; s < s1; ++s) {
    const u64 t = (sl.hi[s] - sl.lo[s] + tile - 1) / tile;
    local += (u32)(t ? t : 1);
  }
  u32 incl = wave_incl_sum(local);
  const u32 w = threadIdx.x >> 6;
  if (__lane_id() == 63) sm[w] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    u32 acc = 0;
    for (int i = 0; i < 16; ++i) {
      u32 t = sm[i];
      sm[i] = acc;
      acc += t;
    }
    sm[16] = acc;
  }
  __syncthreads();
  u32 run = sm[w] + incl - local;
  for (u32 s = s0; s < s1; ++s) {
    tile_start[s] = run;
    const u64 t = (sl.hi[s] - sl.lo[s] + tile - 1) / tile;
    run += (u32)(t ? t : 1);
  }
  if (threadIdx.x == 0) tile_start[n_seg] = sm[16];
}

kpa_status launch_seg_tiles_list(const SegList& sl, u32 tile, u32* tile_start, hipStream_t st) {
  KPA_LAUNCH("seg_tiles", k_seg_tiles_list, dim3(1), dim3(1024), 0, st, sl, tile, tile_start);
  return KPA_OK;
}

kpa_status radix_sort_plan(u64 n_cap, u32 n_seg, Carver& c, RadixWs* w, bool vals, bool tmp) {
  const u64 tiles = max_tiles(n_cap, n_seg, TILE);
  w->keys_tmp = tmp ? c.take<u64>(n_cap) : nullptr;
  w->rids_tmp = tmp ? c.take<u32>(n_cap) : nullptr;
  w->vals_tmp = tmp && vals ? c.take<u64>(n_cap) : nullptr;
  w->hist = c.take<u32>((u64)n_seg * 8 * RADIX);
  w->seg_mask = c.take<u32>(n_seg);
  w->tile_start = c.take<u32>((u64)n_seg + 1);
  w->status0 = c.take<u32>(tiles * RADIX);
  w->status1 = c.take<u32>(tiles * RADIX);
  w->counters = c.take<u32>(16);
  order_plan(c, tiles, n_seg, &w->order);
  w->max_tiles = tiles;
  w->max_seg = n_seg;
  return KPA_OK;
}

kpa_status radix_sort_launch(const u64* keys_in, const u32* rids_in, u64* keys_out,
                             u32* rids_out, const SegList& sl, const RadixWs& w,
                             hipStream_t st, u64* unsupported, const u64* vals_in,
                             u64* vals_out) {
  KPA_REQUIRE(!vals_in || (vals_out && w.vals_tmp), KPA_EINVAL,
              "a value column needs an output and a planned buffer");
  DigitSortBufs b{keys_in,    rids_in,       keys_out,   rids_out,  w.keys_tmp,
                  w.rids_tmp, w.hist,        w.seg_mask, w.tile_start, w.status0,
                  w.status1,  w.counters,    w.max_tiles, w.order, unsupported,
                  vals_in,    vals_in ? vals_out : nullptr, vals_in ? w.vals_tmp : nullptr};
  return digit_sort_launch<RadixDF>(sl, RadixDF::Params{}, b, st);
}

kpa_status radix_sort_inplace(u64* keys, u32* rids, u64* vals, const SegList& sl,
                              const RadixWs& w, u64* tmp_k, u32* tmp_r, u64* tmp_v,
                              hipStream_t st, u64* unsupported) {
  KPA_REQUIRE(tmp_k && tmp_r && (!vals || tmp_v), KPA_EINVAL, "in-place sort needs scratch");
  DigitSortBufs b{keys,  rids,   keys,       rids,          tmp_k,     tmp_r,
                  w.hist, w.seg_mask, w.tile_start, w.status0, w.status1, w.counters,
                  w.max_tiles, w.order, unsupported, vals, vals, vals ? tmp_v : nullptr, true};
  return digit_sort_launch<RadixDF>(sl, RadixDF::Params{}, b, st);
}

}  // namespace kpa
