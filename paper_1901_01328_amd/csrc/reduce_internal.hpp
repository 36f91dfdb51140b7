// Keyed reduction internals shared by reduce, median and join.
#pragma once

#include "kpa_internal.hpp"

namespace kpa {

// Aggregate of a (partial) run of equal keys.  f: the run contains its head.
struct SegAgg {
  u32 f;
  u64 c, s, m, hp;  // count, sum (mod 2^64), max, global index of the head
};

__device__ __forceinline__ SegAgg seg_identity() { return SegAgg{0u, 0ull, 0ull, 0ull, 0ull}; }

// Segmented-scan operator: b continues a unless b starts a new run.
__device__ __forceinline__ SegAgg seg_combine(const SegAgg& a, const SegAgg& b) {
  if (b.f) return b;
  return SegAgg{a.f, a.c + b.c, a.s + b.s, a.m > b.m ? a.m : b.m, a.hp};
}

struct ReduceWs {
  u32* tile_start;
  u32* tile_seg;  // segment of each tile
  u32* heads;   // runs starting in each tile
  u32* flags;   // bit 0: the tile's last run continues into the next tile
  u64* gbase;   // groups started before each tile
  u64* bsum;    // scan blocks: group counts, then their exclusive prefix
  u64 max_tiles;
};

struct ReduceOut {
  u64* gkey;
  u64* cnt;
  u64* sum;
  u64* max;
  u64* gstart;
  u64* gseg_off;
};

void reduce_plan(u64 n_cap, u32 n_seg, Carver& c, ReduceWs* w);

// Exclusive prefix over the tiles of a tile map of per-tile counts (one u32
// per tile): tbase[t] = sum of counts of tiles before t, seg_first[s] =
// tbase of segment s's first tile, seg_first[n_seg] = the total.  bsum holds
// ceil(max_tiles / 1024) u64.
constexpr u32 SCAN_TILES = 1024;
kpa_status launch_tile_scan(const u32* counts, const u32* tile_start, const u32* tile_seg,
                            u32 n_seg, u64 max_tiles, u64* bsum, u64* tbase, u64* seg_first,
                            hipStream_t st);
kpa_status reduce_launch(const u64* keys, const u32* rids, const u64* seg_off, u32 n_seg,
                         const unsigned char* rows, const kpa_row_layout* L, bool need_val,
                         const ReduceOut& o, const ReduceWs& w, hipStream_t st);

}  // namespace kpa
