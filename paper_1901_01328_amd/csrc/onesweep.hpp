// One stable counting-scatter pass over a tile of 4096 entries with 256
// digits, in the single-pass ("onesweep") form: the tile ranks its entries by
// digit in on-chip memory, publishes its per-digit counts, obtains the counts
// of all earlier tiles of its segment by decoupled look-back (Merrill &
// Garland 2016; Adinets & Merrill 2022), then writes its entries through an
// LDS staging buffer so that each digit's run goes out as one contiguous
// stretch.  Used by the window partition (digit = window) and by every radix
// pass (digit = 8 key bits).
#pragma once

#include "kpa_internal.hpp"

namespace kpa {

constexpr int RADIX = 256;
static_assert(RADIX == BLOCK, "one thread per digit");

struct OnesweepSmem {
  u32 whist[WAVES][RADIX];  // per-wave running digit counts, then per-wave offsets
  u32 lstart[RADIX];        // first LDS slot of each digit in the tile
  u64 gbase[RADIX];         // global destination of each digit's first entry of the tile
  u32 scan[WAVES + 1];
  u32 tile;
  u32 count;
  u64 skeys[TILE];
  u32 srids[TILE];
  unsigned char sdig[TILE];
};

// Entry (wave w, item j, lane l) sits at tile offset w*64*ITEMS + j*64 + l:
// each wave owns a contiguous quarter of the tile and loads it coalesced.
__device__ __forceinline__ u32 tile_offset(int j) {
  return (threadIdx.x >> 6) * (64 * ITEMS) + j * 64 + __lane_id();
}

// Ranks, publishes, looks back and scatters.  k/r/d hold this thread's items;
// item j is present iff bit j of `valid` is set.  my_digit_base is, for the
// digit equal to this thread's index, the global index where that digit of
// the segment begins (segment start plus the segment's exclusive digit count).  status points at the look-back words of
// tile 0; the tile's own row is status + tile*RADIX.  first: the tile is the
// first of its segment (its prefix is its own count).
__device__ __forceinline__ void onesweep_tile(OnesweepSmem& sm, const u64 (&k)[ITEMS],
                                              const u32 (&r)[ITEMS], const u32 (&d)[ITEMS],
                                              u32 valid, u32* __restrict__ status, u32 tile,
                                              bool first, u64 my_digit_base,
                                              u64* __restrict__ keys_out,
                                              u32* __restrict__ rids_out) {
  const u32 tid = threadIdx.x;
  const u32 w = tid >> 6;
  const u32 lane = __lane_id();
  u32* wh = sm.whist[w];
#pragma unroll
  for (int i = 0; i < RADIX / 64; ++i) wh[lane + 64 * i] = 0;

  // Stable rank within the wave, item by item: lanes holding the same digit
  // ("peers") are found with one ballot per digit bit.
  u32 rank[ITEMS];
  const u64 lt = lanemask_lt();
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const bool v = (valid >> j) & 1;
    const u32 dj = d[j];
    u64 peers = ballot(v);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (dj >> b) & 1;
      const u64 bal = ballot(bit);
      peers &= bit ? bal : ~bal;
    }
    u32 before = wh[dj];
    const u32 below = (u32)__popcll(peers & lt);
    if (v && below == 0) wh[dj] = before + (u32)__popcll(peers);
    rank[j] = before + below;
  }
  __syncthreads();

  // Thread t owns digit t: per-wave exclusive offsets and the tile's count.
  u32 c0 = sm.whist[0][tid], c1 = sm.whist[1][tid], c2 = sm.whist[2][tid], c3 = sm.whist[3][tid];
  sm.whist[0][tid] = 0;
  sm.whist[1][tid] = c0;
  sm.whist[2][tid] = c0 + c1;
  sm.whist[3][tid] = c0 + c1 + c2;
  const u32 total = c0 + c1 + c2 + c3;
  u32* my = status + (u64)tile * RADIX + tid;
  st_status(my, (first ? ST_PRE : ST_AGG) | total);

  u32 tile_count;
  const u32 ls = block_excl_sum(total, sm.scan, &tile_count);
  sm.lstart[tid] = ls;

  // Decoupled look-back over earlier tiles of the segment.  Every tile with a
  // lower index was claimed by a running workgroup before this one and
  // publishes its count without waiting, so the loop ends.
  u32 excl = 0;
  if (!first) {
    const u32* p = my - RADIX;
    while (true) {
      u32 s;
      s = ld_status(p);
      while ((s & ~ST_VAL) == 0) {
        __builtin_amdgcn_s_sleep(1);
        s = ld_status(p);
      }
      excl += s & ST_VAL;
      if (s & ST_PRE) break;
      p -= RADIX;
    }
    st_status(my, ST_PRE | (excl + total));
  }
  sm.gbase[tid] = my_digit_base + excl;
  if (tid == 0) sm.count = tile_count;
  __syncthreads();

  // Stage the tile in digit order.
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    if ((valid >> j) & 1) {
      const u32 pos = sm.lstart[d[j]] + sm.whist[w][d[j]] + rank[j];
      sm.skeys[pos] = k[j];
      sm.srids[pos] = r[j];
      sm.sdig[pos] = (unsigned char)d[j];
    }
  }
  __syncthreads();

  const u32 n = sm.count;
  for (u32 i = tid; i < n; i += BLOCK) {
    const u32 dd = sm.sdig[i];
    const u64 dst = sm.gbase[dd] + (i - sm.lstart[dd]);
    keys_out[dst] = sm.skeys[i];
    rids_out[dst] = sm.srids[i];
  }
}

}  // namespace kpa
