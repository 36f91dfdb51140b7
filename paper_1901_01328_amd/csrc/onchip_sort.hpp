// Stable sort of up to one tile (4096 entries) held in on-chip memory, and the
// block-wide reductions it uses.  Shared by the learned sort's finishing pass
// and the batched small-segment path.
#pragma once

#include "onesweep.hpp"

namespace kpa {

// Block-wide reductions over NW waves (sm: NW u32, resp. 2*NW u64).
template <int NW = WAVES>
__device__ __forceinline__ u32 block_min_u32(u32 v, u32* sm) {
  v = wave_reduce(v, 0xFFFFFFFFu, [](u32 a, u32 b) { return a < b ? a : b; });
  __syncthreads();
  if (__lane_id() == 0) sm[threadIdx.x >> 6] = v;
  __syncthreads();
  u32 r = sm[0];
  for (int i = 1; i < NW; ++i) r = sm[i] < r ? sm[i] : r;
  __syncthreads();
  return r;
}

template <int NW = WAVES>
__device__ __forceinline__ void block_or_and(u64& o, u64& a, u64* sm) {
  o = wave_reduce(o, (u64)0, [](u64 x, u64 y) { return x | y; });
  a = wave_reduce(a, ~(u64)0, [](u64 x, u64 y) { return x & y; });
  __syncthreads();
  if (__lane_id() == 0) {
    sm[threadIdx.x >> 6] = o;
    sm[NW + (threadIdx.x >> 6)] = a;
  }
  __syncthreads();
  o = sm[0];
  a = sm[NW];
  for (int i = 1; i < NW; ++i) {
    o |= sm[i];
    a &= sm[NW + i];
  }
  __syncthreads();
}

constexpr u32 NONE = 0xFFFFFFFFu;

// Stable sort of the m <= SM::kWaves*64 entries in sm.skeys/sm.srids [0, m)
// by counting: thread t takes entry t and counts the entries that precede it
// (smaller key, or equal key at a lower position); all threads read the same
// key at the same time, so each read is one LDS broadcast.  Returns false
// when the entries were already in order (nothing moved).
template <class SM>
__device__ bool rank_sort_small(SM& sm, u32 m) {
  const u32 tid = threadIdx.x;
  __syncthreads();
  const bool mine = tid < m;
  u64 k = 0;
  u32 r = 0, rank = 0;
  if (mine) {
    k = sm.skeys[tid];
    r = sm.srids[tid];
    for (u32 q = 0; q < m; ++q) {
      const u64 kq = sm.skeys[q];
      rank += (kq < k) || (kq == k && q < tid);
    }
  }
  const bool moved = __syncthreads_or(mine && rank != tid);
  if (moved && mine) {
    sm.skeys[rank] = k;
    sm.srids[rank] = r;
  }
  __syncthreads();
  return moved;
}

// Stable on-chip sort of the m <= TILE entries held in sm.skeys/sm.srids
// [0, m) by a workgroup of SM::kWaves waves: LSD over the bytes that vary
// among the keys, one rank-and-move per byte, data kept in LDS between
// passes.  Returns with the sorted entries in sm (and false when nothing
// varied).
template <class SM>
__device__ bool lds_sort(SM& sm, u32 m) {
  constexpr int NW = SM::kWaves;
  constexpr int IT = TILE / (64 * NW);
  const u32 tid = threadIdx.x;
  const u32 w = tid >> 6;
  __syncthreads();
  u64 vor = 0, vand = ~0ull;
  for (u32 i = tid; i < m; i += NW * 64) {
    vor |= sm.skeys[i];
    vand &= sm.skeys[i];
  }
  block_or_and<NW>(vor, vand, sm.red64);
  const u64 vary = vor ^ vand;
  if (vary == 0) return false;
  u32 valid = 0;
#pragma unroll
  for (int j = 0; j < IT; ++j)
    if (part_offset<NW, IT>(j) < m) valid |= 1u << j;
#pragma unroll 1
  for (u32 p = 0; p < 8; ++p) {
    if (((vary >> (8 * p)) & 255u) == 0) continue;
    u64 kk[IT];
    u32 rr[IT], d[IT], rank[IT], tc;
#pragma unroll
    for (int j = 0; j < IT; ++j) {
      const u32 o = part_offset<NW, IT>(j);
      kk[j] = ((valid >> j) & 1) ? sm.skeys[o] : 0ull;
      rr[j] = ((valid >> j) & 1) ? sm.srids[o] : 0u;
      d[j] = (u32)(kk[j] >> (8 * p)) & 255u;
    }
    // every thread has read its items before rank_tile's first barrier; the
    // scatter below may overwrite them after its last one
    rank_tile(sm.whist, sm.lstart, sm.scan, d, valid, rank, &tc);
#pragma unroll
    for (int j = 0; j < IT; ++j)
      if ((valid >> j) & 1) {
        const u32 pos = sm.lstart[d[j]] + sm.whist[w][d[j]] + rank[j];
        sm.skeys[pos] = kk[j];
        sm.srids[pos] = rr[j];
      }
    __syncthreads();
  }
  return true;
}

}  // namespace kpa
