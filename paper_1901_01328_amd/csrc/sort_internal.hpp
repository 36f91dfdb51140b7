// Workspace layouts and launch entry points shared between the sort files.
#pragma once

#include "onesweep.hpp"

namespace kpa {

constexpr u32 SEG_UNSUPPORTED = 1u << 31;

// Segments [lo[s], hi[s]) for s < n, n = *n_dev when n_dev is set (a count
// produced on the device), else n_max.
struct SegList {
  const u64* lo;
  const u64* hi;
  const u32* n_dev;
  u32 n_max;
  __device__ __forceinline__ u32 n() const { return n_dev ? min(*n_dev, n_max) : n_max; }
};

inline SegList seg_list_from_offsets(const u64* off, u32 n_seg) {
  return SegList{off, off + 1, nullptr, n_seg};
}

// tile_start[s] = sum over s' < s of max(1, ceil(len(s')/tile)); tile_start[n] = total.
kpa_status launch_seg_tiles_list(const SegList& sl, u32 tile, u32* tile_start, hipStream_t st);

// One claimable tile of a scatter pass: where its entries are and which
// look-back row (g, the tile's index in the segment-major tile map) it uses.
struct TileDesc {
  u64 base;   // first entry
  u32 seg;
  u32 t_in;   // tile index within the segment
  u32 cnt;    // entries (0 for the one tile of an empty segment)
  u32 g;      // tile_start[seg] + t_in
  u32 mask;   // the segment's pass mask
  u32 pad;
};

// Claim order of the scatter passes: round r holds tile r of every segment
// that has more than r tiles, so that the workgroups in flight spread over
// the segments and each segment's tiles are still claimed in order.
struct OrderBufs {
  TileDesc* desc;  // max_tiles, in claim order
  u32* more;       // more[r] = segments with more than r tiles (max_tiles + 2)
  u32* round0;     // round0[r] = first claim index of round r (max_tiles + 2)
  u32* ties;       // per tile count: next position among equal segments (max_tiles + 2)
  u32* pos;        // n_seg: position of the segment inside every round
  // Per pass p (up to LIST_PASSES): the claim indices of the tiles whose
  // segment is sorted in pass p, in claim order (lists + p*max_tiles), and
  // per LIST_BLK claims their count, then offset; entry nblk: the list size.
  u32* lists;
  u32* lcount;  // LIST_PASSES * (nblk + 1)
};

constexpr int LIST_PASSES = 8;
constexpr u32 LIST_BLK = 1024;  // claims per list-building workgroup
__host__ __device__ inline u64 list_blocks(u64 max_tiles) { return (max_tiles + LIST_BLK - 1) / LIST_BLK; }

inline void order_plan(Carver& c, u64 max_tiles, u32 n_seg, OrderBufs* o) {
  o->desc = c.take<TileDesc>(max_tiles);
  o->more = c.take<u32>(max_tiles + 2);
  o->round0 = c.take<u32>(max_tiles + 2);
  o->ties = c.take<u32>(max_tiles + 2);
  o->pos = c.take<u32>(n_seg);
  o->lists = c.take<u32>((u64)LIST_PASSES * max_tiles);
  o->lcount = c.take<u32>((u64)LIST_PASSES * (list_blocks(max_tiles) + 1));
}

struct RadixDigit {
  u32 shift;
  __device__ __forceinline__ u32 operator()(u64 k) const { return (u32)(k >> shift) & 255u; }
};

struct RadixWs {
  u64* keys_tmp;
  u32* rids_tmp;
  u64* vals_tmp;    // planned with a value column only (else null)
  u32* hist;        // n_seg * 8 * 256: digit counts, then exclusive offsets
  u32* seg_mask;    // n_seg: bit p set when pass p is needed
  u32* tile_start;  // n_seg + 1
  u32* status0;     // look-back words, max_tiles * 256, two alternating buffers
  u32* status1;
  u32* counters;    // 16 tile counters (one per pass; [15]: passes needed by any segment)
  OrderBufs order;
  u64 max_tiles;
  u32 max_seg;
};

// vals: also plan the ping-pong buffer of a value column; tmp = false: no
// ping-pong buffers at all (for radix_sort_inplace, which borrows them).
kpa_status radix_sort_plan(u64 n_cap, u32 n_seg, Carver& c, RadixWs* w, bool vals = false,
                           bool tmp = true);
// unsupported (device, may be null): counts the entries of segments of 2^30
// or more entries, which are copied through unsorted.  vals_in/vals_out
// (both or neither; the plan must have had vals): a value column that
// follows the keys' permutation.
kpa_status radix_sort_launch(const u64* keys_in, const u32* rids_in, u64* keys_out,
                             u32* rids_out, const SegList& sl, const RadixWs& w, hipStream_t st,
                             u64* unsupported = nullptr, const u64* vals_in = nullptr,
                             u64* vals_out = nullptr);
// Sorts the segments of sl in place in keys/rids (and vals, may be null),
// with tmp_* (n_cap each, the caller's scratch) as the ping-pong partner: a
// segment with an odd number of active passes is first copied there.  The
// plan may have been made with tmp = false.
kpa_status radix_sort_inplace(u64* keys, u32* rids, u64* vals, const SegList& sl,
                              const RadixWs& w, u64* tmp_k, u32* tmp_r, u64* tmp_v,
                              hipStream_t st, u64* unsupported = nullptr);
// Offset of kpa_sort_stats.unsupported_entries in u64 words; the struct's size.
constexpr int STATS_UNSUPPORTED = 6;
constexpr int STATS_WORDS = 7;
inline u64* stats_unsupported(kpa_sort_stats* st) {
  return st ? reinterpret_cast<u64*>(st) + STATS_UNSUPPORTED : nullptr;
}

}  // namespace kpa
