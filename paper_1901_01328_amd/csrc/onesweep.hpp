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
#ifndef KPA_LB_WINDOW
#define KPA_LB_WINDOW 4
#endif
constexpr int LB_WINDOW = KPA_LB_WINDOW;  // look-back tiles probed per round trip
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

// Stable rank of a tile's entries by digit.  Item j of this thread (tile
// offset tile_offset(j)) is present iff bit j of `valid` is set.  On return:
// rank[j] = position of item j among the tile's entries with the same digit
// that precede it in the wave, whist[w][d] = entries with digit d in waves
// before w, lstart[d] = entries of the tile with a smaller digit, and the
// return value is this thread's digit (d = threadIdx.x) count in the tile.
// *tile_count receives the number of present entries.  Lanes holding the same
// digit ("peers") are found with one ballot per digit bit.
__device__ __forceinline__ u32 rank_tile(u32 (&whist)[WAVES][RADIX], u32* lstart, u32* scan,
                                         const u32 (&d)[ITEMS], u32 valid, u32 (&rank)[ITEMS],
                                         u32* tile_count) {
  const u32 tid = threadIdx.x;
  const u32 w = tid >> 6;
  const u32 lane = __lane_id();
  u32* wh = whist[w];
#pragma unroll
  for (int i = 0; i < RADIX / 64; ++i) wh[lane + 64 * i] = 0;
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
  const u32 c0 = whist[0][tid], c1 = whist[1][tid], c2 = whist[2][tid], c3 = whist[3][tid];
  whist[0][tid] = 0;
  whist[1][tid] = c0;
  whist[2][tid] = c0 + c1;
  whist[3][tid] = c0 + c1 + c2;
  const u32 total = c0 + c1 + c2 + c3;
  lstart[tid] = block_excl_sum(total, scan, tile_count);
  return total;
}

// Moves a ranked tile (rank_tile's outputs still in sm.whist/sm.lstart)
// through LDS in digit order, then writes each digit's entries contiguously
// from sm.gbase[digit].  The caller has set sm.gbase and sm.count and passed
// a barrier since.
template <class SM>
__device__ __forceinline__ void stage_scatter(SM& sm, const u64 (&k)[ITEMS], const u32 (&r)[ITEMS],
                                              const u32 (&d)[ITEMS], const u32 (&rank)[ITEMS],
                                              u32 valid, u64* __restrict__ keys_out,
                                              u32* __restrict__ rids_out) {
  const u32 tid = threadIdx.x;
  const u32 w = tid >> 6;
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
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const u32 i = tid + j * BLOCK;
    if (i < n) {
      const u32 dd = sm.sdig[i];
      const u64 dst = sm.gbase[dd] + (i - sm.lstart[dd]);
      keys_out[dst] = sm.skeys[i];
      rids_out[dst] = sm.srids[i];
    }
  }
}

// Ranks, publishes, looks back and scatters.  k/r/d hold this thread's items;
// item j is present iff bit j of `valid` is set.  my_digit_base is, for the
// digit equal to this thread's index, the global index where that digit of
// the segment begins (segment start plus the segment's exclusive digit count).
// status points at the look-back words of tile 0; the tile's own row is
// status + tile*RADIX.  tile_in_seg: index of the tile within its segment (the
// first tile's prefix is its own count).
__device__ __forceinline__ void onesweep_tile(OnesweepSmem& sm, const u64 (&k)[ITEMS],
                                              const u32 (&r)[ITEMS], const u32 (&d)[ITEMS],
                                              u32 valid, u32* __restrict__ status, u32 tile,
                                              u32 tile_in_seg, u64 my_digit_base,
                                              u64* __restrict__ keys_out,
                                              u32* __restrict__ rids_out) {
  const u32 tid = threadIdx.x;
  const u32 w = tid >> 6;
  const bool first = tile_in_seg == 0;
  u32 rank[ITEMS];
  u32 tile_count;
  // Publish the tile's counts as soon as they are known (inside rank_tile the
  // counts are complete before the block scan).
  const u32 total = rank_tile(sm.whist, sm.lstart, sm.scan, d, valid, rank, &tile_count);
  u32* my = status + (u64)tile * RADIX + tid;
  if (first) st_status(my, ST_PRE | total);
  else st_status(my, ST_AGG | total);

  // Decoupled look-back over earlier tiles of the segment, LB_WINDOW tiles
  // per round trip.  Every tile with a lower index was claimed by a running
  // workgroup before this one and publishes its count without waiting, so the
  // loop ends; the segment's first tile always holds a prefix.
  u32 excl = 0;
  if (!first) {
    const u32* p = my - RADIX;
    u32 left = tile_in_seg;  // predecessors in the segment
    while (true) {
      u32 s[LB_WINDOW];
#pragma unroll
      for (int i = 0; i < LB_WINDOW; ++i) s[i] = (u32)i < left ? ld_status(p - i * RADIX) : ST_PRE;
      u32 acc = 0, used = 0;
      bool done = false, stalled = false;
#pragma unroll
      for (int i = 0; i < LB_WINDOW; ++i) {
        if (!done && !stalled) {
          if ((s[i] & ~ST_VAL) == 0) {
            stalled = true;
          } else {
            acc += s[i] & ST_VAL;
            ++used;
            if (s[i] & ST_PRE) done = true;
          }
        }
      }
      excl += acc;
      if (done) break;
      p -= used * RADIX;
      left -= used;
      if (stalled) __builtin_amdgcn_s_sleep(1);
    }
    st_status(my, ST_PRE | (excl + total));
  }
  sm.gbase[tid] = my_digit_base + excl;
  if (tid == 0) sm.count = tile_count;
  __syncthreads();

  stage_scatter(sm, k, r, d, rank, valid, keys_out, rids_out);
}

}  // namespace kpa
