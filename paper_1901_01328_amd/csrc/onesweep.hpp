// One stable counting-scatter pass over a tile of 4096 entries with 256
// digits, in the single-pass ("onesweep") form: the tile ranks its entries by
// digit in on-chip memory, publishes its per-digit counts, obtains the counts
// of all earlier tiles of its segment by decoupled look-back (Merrill &
// Garland 2016; Adinets & Merrill 2022), then writes its entries through an
// LDS staging buffer so that each digit's run goes out as one contiguous
// stretch.  Used by the window partition (digit = window) and by every radix
// pass (digit = 8 key bits).
//
// The routines are templates over the workgroup's wave count NW: a tile is
// always TILE entries, spread over NW*64 threads with TILE/(NW*64) items each.
// Threads 0..255 own one digit each in the per-digit steps.
#pragma once

#include "kpa_internal.hpp"

namespace kpa {

constexpr int RADIX = 256;
#ifndef KPA_LB_WINDOW
#define KPA_LB_WINDOW 4
#endif
constexpr int LB_WINDOW = KPA_LB_WINDOW;  // look-back tiles probed per round trip
static_assert(RADIX == BLOCK, "one thread per digit in 256-thread workgroups");

template <int NW>
struct OnesweepSmemT {
  u32 whist[NW][RADIX];  // per-wave running digit counts, then per-wave offsets
  u32 lstart[RADIX];     // first LDS slot of each digit in the tile
  u64 gbase[RADIX];      // global destination of each digit's first entry of the tile
  u32 scan[NW + 1];
  u32 tile;
  u32 count;
  u64 skeys[TILE];
  u32 srids[TILE];
  unsigned char sdig[TILE];
};
using OnesweepSmem = OnesweepSmemT<WAVES>;

// Entry (wave w, item j, lane l) sits at tile offset w*64*IT + j*64 + l with
// IT = TILE/(NW*64): each wave owns a contiguous part of the tile and loads it
// coalesced.
template <int NW>
__device__ __forceinline__ u32 tile_offset_t(int j) {
  return (threadIdx.x >> 6) * (TILE / NW) + j * 64 + __lane_id();
}
__device__ __forceinline__ u32 tile_offset(int j) { return tile_offset_t<WAVES>(j); }

// The same layout for a part of a tile: NW waves of IT items each, wave w
// owning entries [w*64*IT, (w+1)*64*IT).
template <int NW, int IT>
__device__ __forceinline__ u32 part_offset(int j) {
  return (threadIdx.x >> 6) * (64 * IT) + j * 64 + __lane_id();
}

// First half of the stable rank: lanes holding the same digit ("peers") are
// found with one ballot per digit bit; rank[j] = position of item j among the
// tile's entries with the same digit that precede it in its wave.  Threads
// t < 256 then turn column t into whist[w][t] = entries with digit t in waves
// before w and get the tile's count of digit t (0 for other threads); the
// caller synchronizes before any thread reads another thread's column.
// Item j is present iff bit j of `valid` is set.  Items are laid out as in
// part_offset<NW, IT> (for NW*64*IT == TILE, as in tile_offset_t<NW>).  Every
// digit is below 2^nbits (nbits uniform over the workgroup): only those bits
// are matched.
template <int NW, int IT>
__device__ __forceinline__ u32 rank_count(u32 (&whist)[NW][RADIX], const u32 (&d)[IT], u32 valid,
                                          u32 (&rank)[IT], u32 nbits = 8) {
  static_assert(NW * 64 * IT <= TILE && IT <= 32, "tile geometry");
  const u32 tid = threadIdx.x;
  const u32 w = tid >> 6;
  const u32 lane = __lane_id();
  u32* wh = whist[w];
#pragma unroll
  for (int i = 0; i < RADIX / 64; ++i) wh[lane + 64 * i] = 0;
  const u64 lt = lanemask_lt();
#pragma unroll
  for (int j = 0; j < IT; ++j) {
    const bool v = (valid >> j) & 1;
    const u32 dj = d[j];
    u64 peers = ballot(v);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      if ((u32)b < nbits) {
        const bool bit = (dj >> b) & 1;
        const u64 bal = ballot(bit);
        peers &= bit ? bal : ~bal;
      }
    }
    u32 before = wh[dj];
    const u32 below = (u32)__popcll(peers & lt);
    if (v && below == 0) wh[dj] = before + (u32)__popcll(peers);
    rank[j] = before + below;
  }
  __syncthreads();
  u32 total = 0;
  if (tid < RADIX) {
#pragma unroll
    for (int w2 = 0; w2 < NW; ++w2) {
      const u32 c = whist[w2][tid];
      whist[w2][tid] = total;
      total += c;
    }
  }
  return total;
}

// Second half: lstart[d] = entries of the tile with a smaller digit;
// *tile_count = present entries.  The 256 digit counts sit in the first four
// waves: each scans its 64 in registers, then adds the totals of the waves
// before it (two barriers in all; ends with one).
template <int NW>
__device__ __forceinline__ void rank_starts(u32 total, u32* lstart, u32* scan, u32* tile_count) {
  static_assert(NW * 64 >= RADIX && RADIX == 256, "digit counts span four waves");
  const u32 tid = threadIdx.x, w = tid >> 6;
  u32 incl = 0;
  if (tid < RADIX) {  // whole waves
    incl = wave_incl_sum(total);
    if (__lane_id() == 63) scan[w] = incl;
  }
  __syncthreads();
  const u32 s0 = scan[0], s1 = scan[1], s2 = scan[2], s3 = scan[3];
  if (tid < RADIX) lstart[tid] = (w > 0 ? s0 : 0u) + (w > 1 ? s1 : 0u) + (w > 2 ? s2 : 0u) + incl - total;
  *tile_count = s0 + s1 + s2 + s3;
  __syncthreads();
}

// Both halves (for callers that do not publish in between).
template <int NW, int IT>
__device__ __forceinline__ u32 rank_tile(u32 (&whist)[NW][RADIX], u32* lstart, u32* scan,
                                         const u32 (&d)[IT], u32 valid, u32 (&rank)[IT],
                                         u32* tile_count, u32 nbits = 8) {
  const u32 total = rank_count<NW, IT>(whist, d, valid, rank, nbits);
  rank_starts<NW>(total, lstart, scan, tile_count);
  return total;
}

// Moves a ranked tile into LDS in digit order (stable).  Ends with a barrier.
template <class SM, int IT>
__device__ __forceinline__ void stage_tile(SM& sm, const u64 (&k)[IT], const u32 (&r)[IT],
                                           const u32 (&d)[IT], const u32 (&rank)[IT],
                                           u32 valid) {
  const u32 w = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < IT; ++j) {
    if ((valid >> j) & 1) {
      const u32 pos = sm.lstart[d[j]] + sm.whist[w][d[j]] + rank[j];
      sm.skeys[pos] = k[j];
      sm.srids[pos] = r[j];
      sm.sdig[pos] = (unsigned char)d[j];
    }
  }
  __syncthreads();
}

// stage_tile that also returns each present item's LDS slot (pos), for a
// second round that moves a value column through the same slots.
template <class SM, int IT>
__device__ __forceinline__ void stage_tile_pos(SM& sm, const u64 (&k)[IT], const u32 (&r)[IT],
                                               const u32 (&d)[IT], const u32 (&rank)[IT],
                                               u32 valid, u32 (&pos)[IT]) {
  const u32 w = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < IT; ++j) {
    pos[j] = 0;
    if ((valid >> j) & 1) {
      pos[j] = sm.lstart[d[j]] + sm.whist[w][d[j]] + rank[j];
      sm.skeys[pos[j]] = k[j];
      sm.srids[pos[j]] = r[j];
      sm.sdig[pos[j]] = (unsigned char)d[j];
    }
  }
  __syncthreads();
}

// Second round of a staged tile: after its keys and row ids are written
// (write_staged), the items' values go through the key slots of LDS to the
// same destinations.  pos: the slots stage_tile_pos returned.  Begins with a
// barrier (every thread has read the staged keys) and ends without one.
template <class SM, int NW, int IT>
__device__ __forceinline__ void write_staged_vals(SM& sm, const u64 (&v)[IT], const u32 (&pos)[IT],
                                                  u32 valid, u64* __restrict__ vals_out) {
  constexpr int NT = NW * 64;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < IT; ++j)
    if ((valid >> j) & 1) sm.skeys[pos[j]] = v[j];
  __syncthreads();
  const u32 n = sm.count;
#pragma unroll
  for (int j = 0; j < TILE / NT; ++j) {
    const u32 i = threadIdx.x + j * NT;
    if (i < n) {
      const u32 dd = sm.sdig[i];
      vals_out[sm.gbase[dd] + (i - sm.lstart[dd])] = sm.skeys[i];
    }
  }
}

// Writes the staged tile: each digit's entries contiguously from
// sm.gbase[digit].  The caller has set sm.gbase and sm.count and passed a
// barrier since.
template <class SM, int NW>
__device__ __forceinline__ void write_staged(SM& sm, u64* __restrict__ keys_out,
                                             u32* __restrict__ rids_out) {
  constexpr int NT = NW * 64;
  const u32 n = sm.count;
#pragma unroll
  for (int j = 0; j < TILE / NT; ++j) {
    const u32 i = threadIdx.x + j * NT;
    if (i < n) {
      const u32 dd = sm.sdig[i];
      const u64 dst = sm.gbase[dd] + (i - sm.lstart[dd]);
      keys_out[dst] = sm.skeys[i];
      rids_out[dst] = sm.srids[i];
    }
  }
}

// Stage then write, for callers that know the destinations before staging.
template <class SM, int IT>
__device__ __forceinline__ void stage_scatter(SM& sm, const u64 (&k)[IT], const u32 (&r)[IT],
                                              const u32 (&d)[IT], const u32 (&rank)[IT],
                                              u32 valid, u64* __restrict__ keys_out,
                                              u32* __restrict__ rids_out) {
  stage_tile<SM, IT>(sm, k, r, d, rank, valid);
  write_staged<SM, TILE / (64 * IT)>(sm, keys_out, rids_out);
}

// First half of a tile's scatter: ranks, publishes and stages.  k/r/d hold
// this thread's items; item j is present iff bit j of `valid` is set.
// status points at the look-back words of tile 0; the tile's own row is
// status + tile*RADIX.  tile_in_seg: index of the tile within its segment
// (the first tile's prefix is its own count).  Returns the thread's digit
// count (threads t < 256: digit t) and sets *tile_count; k/r/d are no longer
// needed afterwards.
//
// The tile's counts are published as soon as they are known; the tile is
// staged in LDS before the look-back, so that predecessors have more time to
// publish and the wait overlaps useful work.
template <int NW, int IT>
__device__ __forceinline__ u32 onesweep_rank_stage(OnesweepSmemT<NW>& sm, const u64 (&k)[IT],
                                                   const u32 (&r)[IT], const u32 (&d)[IT],
                                                   u32 valid, u32* __restrict__ status, u32 tile,
                                                   u32 tile_in_seg, u32* tile_count) {
  const u32 tid = threadIdx.x;
  u32 rank[IT];
  const u32 total = rank_count<NW, IT>(sm.whist, d, valid, rank);
  if (tid < RADIX) st_status(status + (u64)tile * RADIX + tid, (tile_in_seg == 0 ? ST_PRE : ST_AGG) | total);
  rank_starts<NW>(total, sm.lstart, sm.scan, tile_count);
  stage_tile<OnesweepSmemT<NW>, IT>(sm, k, r, d, rank, valid);
  return total;
}

// onesweep_rank_stage that also returns the items' LDS slots.
template <int NW, int IT>
__device__ __forceinline__ u32 onesweep_rank_stage_pos(OnesweepSmemT<NW>& sm, const u64 (&k)[IT],
                                                       const u32 (&r)[IT], const u32 (&d)[IT],
                                                       u32 valid, u32* __restrict__ status,
                                                       u32 tile, u32 tile_in_seg,
                                                       u32* tile_count, u32 (&pos)[IT]) {
  const u32 tid = threadIdx.x;
  u32 rank[IT];
  const u32 total = rank_count<NW, IT>(sm.whist, d, valid, rank);
  if (tid < RADIX) st_status(status + (u64)tile * RADIX + tid, (tile_in_seg == 0 ? ST_PRE : ST_AGG) | total);
  rank_starts<NW>(total, sm.lstart, sm.scan, tile_count);
  stage_tile_pos<OnesweepSmemT<NW>, IT>(sm, k, r, d, rank, valid, pos);
  return total;
}

// Second half: decoupled look-back over earlier tiles of the segment, then
// the staged tile goes out.  my_digit_base is, for threads t < 256, the
// global index where digit t of the segment begins (segment start plus the
// segment's exclusive digit count).
//
// The look-back reads LB_WINDOW tiles per round trip.  Every tile with a
// lower index was claimed by a running workgroup before this one and
// publishes its count before waiting on anything, so the loop ends; the
// segment's first tile always holds a prefix.
// The look-back alone: sets sm.gbase (each digit's global destination) and
// sm.count, and ends with a barrier; the caller then writes the staged tile.
template <int NW>
__device__ __forceinline__ void onesweep_lookback(OnesweepSmemT<NW>& sm, u32* __restrict__ status,
                                                  u32 tile, u32 tile_in_seg, u32 total,
                                                  u32 tile_count, u64 my_digit_base) {
  const u32 tid = threadIdx.x;
  if (tid < RADIX) {
    u32* my = status + (u64)tile * RADIX + tid;
    u32 excl = 0;
    if (tile_in_seg != 0) {
      const u32* p = my - RADIX;
      u32 left = tile_in_seg;  // predecessors in the segment
      while (true) {
        u32 s[LB_WINDOW];
#pragma unroll
        for (int i = 0; i < LB_WINDOW; ++i)
          s[i] = (u32)i < left ? ld_status(p - i * RADIX) : ST_PRE;
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
  }
  if (tid == 0) sm.count = tile_count;
  __syncthreads();
}

template <int NW>
__device__ __forceinline__ void onesweep_lookback_write(OnesweepSmemT<NW>& sm,
                                                        u32* __restrict__ status, u32 tile,
                                                        u32 tile_in_seg, u32 total,
                                                        u32 tile_count, u64 my_digit_base,
                                                        u64* __restrict__ keys_out,
                                                        u32* __restrict__ rids_out) {
  onesweep_lookback<NW>(sm, status, tile, tile_in_seg, total, tile_count, my_digit_base);
  write_staged<OnesweepSmemT<NW>, NW>(sm, keys_out, rids_out);
}

// Both halves for one tile.
template <int NW, int IT>
__device__ __forceinline__ void onesweep_tile(OnesweepSmemT<NW>& sm, const u64 (&k)[IT],
                                              const u32 (&r)[IT], const u32 (&d)[IT],
                                              u32 valid, u32* __restrict__ status, u32 tile,
                                              u32 tile_in_seg, u64 my_digit_base,
                                              u64* __restrict__ keys_out,
                                              u32* __restrict__ rids_out) {
  u32 tile_count;
  const u32 total =
      onesweep_rank_stage<NW, IT>(sm, k, r, d, valid, status, tile, tile_in_seg, &tile_count);
  onesweep_lookback_write<NW>(sm, status, tile, tile_in_seg, total, tile_count, my_digit_base,
                              keys_out, rids_out);
}

}  // namespace kpa
