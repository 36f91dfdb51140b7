// Segmented stable LSD sort engine over 8-bit digits produced by a digit
// function DF (key bytes for the radix sort; bytes of a model's bucket id for
// the learned-splitter sort).
//
// DF must provide: PASSES (number of 8-bit digits), SMEM (floats of LDS it
// may use), a Params type, a default constructor, a device constructor
// DF(params, segment), bind(lds) called by all threads before use (then a
// barrier), digit(key, pass) -> [0, 256) and digits(key, d[PASSES]).
#pragma once

#include "sort_internal.hpp"

#include <map>
#include <mutex>
#include <utility>

namespace kpa {

constexpr int HIST_TILES_PER_BLOCK = 8;  // most tiles a histogram workgroup takes at a time

struct DigitSortBufs {
  const u64* keys_in;
  const u32* rids_in;  // may be null: entry i's row id is i
  u64* keys_out;
  u32* rids_out;
  u64* keys_tmp;
  u32* rids_tmp;
  u32* hist;        // n_seg * PASSES * 256
  u32* seg_mask;
  u32* tile_start;
  u32* status0;
  u32* status1;
  u32* counters;    // [p]: tile claims of pass p; [15]: passes needed by any segment
  u64 max_tiles;
  OrderBufs order;
  u64* unsupported;  // may be null: entries of segments too large to sort (copied through)
  // an optional value column carried through the same permutation (all
  // three null when there is none)
  const u64* vals_in = nullptr;
  u64* vals_out = nullptr;
  u64* vals_tmp = nullptr;
  // in place: the data is in the output arrays (keys_in == keys_out); a
  // segment with an even number of passes reads them in its first pass, one
  // with an odd number is first copied to the tmp arrays (k_ds_copy_odd) so
  // that its last pass still lands in the output
  bool in_place = false;
};

__device__ __forceinline__ void seg_tile_range(const SegList& sl, const u32* tile_start,
                                               u32 n_seg, u32 tile, u32& seg, u32& t_in,
                                               u64& a, u64& b, u64& base, u32& cnt,
                                               const u32* tile_seg = nullptr) {
  seg = tile_seg ? tile_seg[tile] : find_seg(tile_start, n_seg, tile);
  t_in = tile - tile_start[seg];
  a = sl.lo[seg];
  b = sl.hi[seg];
  base = a + (u64)t_in * TILE;
  cnt = base < b ? (u32)min<u64>(TILE, b - base) : 0u;
}

// Adds one wave's items to a histogram: the lanes holding the first active
// lane's digit add their count with one atomic (a digit that is constant in
// the segment, or a heavy key, costs one LDS atomic per wave instead of 64
// colliding ones); the other lanes add one each.
__device__ __forceinline__ void wave_hist_add(u32* h, u32 d, bool v) {
  if (v) {
    const u32 d0 = first_lane(d);  // first active lane's digit
    const bool mine = d == d0;
    const u64 same = ballot(mine);  // among the active lanes
    if (mine) {
      if ((same & lanemask_lt()) == 0) atomicAdd(&h[d0], (u32)__popcll(same));
    } else {
      atomicAdd(&h[d], 1u);
    }
  }
}

// Digit counts of every pass per segment: each workgroup takes
// HIST_TILES_PER_BLOCK tiles at a time, loads a tile coalesced (ITEMS per
// thread), counts into per-wave LDS histograms and flushes them with one
// global atomic per nonzero (pass, digit) whenever the segment changes.
template <class DF>
__global__ void __launch_bounds__(BLOCK) k_ds_hist(const u64* __restrict__ keys, SegList sl,
                                                   const u32* __restrict__ tile_start,
                                                   typename DF::Params prm,
                                                   u32* __restrict__ hist, u32 tpb) {
  __shared__ u32 h[WAVES][DF::PASSES][RADIX];
  __shared__ float dfsm[DF::SMEM];
  const u32 tid = threadIdx.x;
  const u32 w = tid >> 6;
  const u32 n_seg = sl.n();
  const u32 total = tile_start[n_seg];
  auto flush = [&](u32 seg) {
    __syncthreads();
    for (int p = 0; p < DF::PASSES; ++p) {
      u32 c = 0;
#pragma unroll
      for (int ww = 0; ww < WAVES; ++ww) {
        c += h[ww][p][tid];
        h[ww][p][tid] = 0;
      }
      if (c) atomicAdd(&hist[((u64)seg * DF::PASSES + p) * RADIX + tid], c);
    }
    __syncthreads();
  };
  for (int p = 0; p < DF::PASSES; ++p)
#pragma unroll
    for (int ww = 0; ww < WAVES; ++ww) h[ww][p][tid] = 0;
  for (u32 t0 = blockIdx.x * tpb; t0 < total; t0 += gridDim.x * tpb) {
    const u32 t1 = min(total, t0 + tpb);
    u32 cur = find_seg(tile_start, n_seg, t0);
    DF df(prm, cur);
    __syncthreads();
    df.bind(dfsm);
    __syncthreads();
    for (u32 t = t0; t < t1; ++t) {
      bool next = false;
      while (cur + 1 < n_seg && tile_start[cur + 1] <= t) {
        flush(cur);
        ++cur;
        next = true;
      }
      if (next) {  // the digit function of the new segment (flush ended with a barrier)
        df = DF(prm, cur);
        df.bind(dfsm);
        __syncthreads();
      }
      const u64 a = sl.lo[cur], b = sl.hi[cur];
      const u64 base = a + (u64)(t - tile_start[cur]) * TILE;
      const u32 cnt = base < b ? (u32)min<u64>(TILE, b - base) : 0u;
      u64 kk[ITEMS];
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) {
        const u32 o = tile_offset(j);
        kk[j] = o < cnt ? keys[base + o] : 0ull;
      }
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) {
        const bool v = tile_offset(j) < cnt;
        u32 dg[DF::PASSES];
        df.digits(kk[j], dg);
#pragma unroll
        for (int p = 0; p < DF::PASSES; ++p) wave_hist_add(h[w][p], dg[p], v);
      }
    }
    flush(cur);
  }
}

// Zeroes what the sort of the device-counted segments needs: their digit
// counts, the first look-back buffer for their tiles, the tile counters.
template <int UNUSED = 0>
__global__ void __launch_bounds__(BLOCK) k_ds_prepare(SegList sl, const u32* __restrict__ tile_start,
                                                      u32* __restrict__ hist, u32 hist_passes,
                                                      u32* __restrict__ status0,
                                                      u32* __restrict__ counters, OrderBufs order,
                                                      u64 max_tiles) {
  const u32 n_seg = sl.n();
  const u64 nh = hist ? (u64)n_seg * hist_passes * RADIX : 0ull;
  const u64 ns = (u64)tile_start[n_seg] * RADIX;
  const u64 stride = (u64)gridDim.x * BLOCK;
  for (u64 i = (u64)blockIdx.x * BLOCK + threadIdx.x; i < nh; i += stride) hist[i] = 0;
  for (u64 i = (u64)blockIdx.x * BLOCK + threadIdx.x; i < ns; i += stride) status0[i] = 0;
  for (u64 i = (u64)blockIdx.x * BLOCK + threadIdx.x; i < max_tiles + 2; i += stride) {
    order.more[i] = 0;
    order.ties[i] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x < 16) counters[threadIdx.x] = 0;
}

// One workgroup per segment: counts -> exclusive offsets, and the mask of the
// passes whose digit varies within the segment.
template <class DF>
__global__ void __launch_bounds__(BLOCK) k_ds_scan(SegList sl, u32* __restrict__ hist,
                                                   u32* __restrict__ seg_mask,
                                                   u64* __restrict__ unsupported) {
  __shared__ u32 sc[WAVES + 1];
  const u32 n_seg = sl.n();
  for (u32 s = blockIdx.x; s < n_seg; s += gridDim.x) {
    const u64 n = sl.hi[s] - sl.lo[s];
    u32 mask = 0;
    for (u32 p = 0; p < (u32)DF::PASSES; ++p) {
      u32* hp = hist + ((u64)s * DF::PASSES + p) * RADIX;
      const u32 c = hp[threadIdx.x];
      u32 tot;
      const u32 ex = block_excl_sum(c, sc, &tot);
      hp[threadIdx.x] = ex;
      const int constant = __syncthreads_or(c == n);
      if (!constant) mask |= 1u << p;
    }
    // Segments of 2^30 or more entries exceed the look-back word; they are
    // copied through unsorted (mask bit 31) and counted, rather than sorted
    // wrongly.
    if (threadIdx.x == 0) {
      seg_mask[s] = n >= MAX_SEG_ENTRIES ? SEG_UNSUPPORTED : mask;
      if (n >= MAX_SEG_ENTRIES && unsupported)
        atomicAdd(reinterpret_cast<unsigned long long*>(unsupported), (unsigned long long)n);
    }
    __syncthreads();
  }
}

// Persistent: each workgroup claims tiles in increasing order until none is
// left.  A tile only waits (look-back) on tiles claimed earlier by running
// workgroups, so every wait ends.
// Claim order, step 1: more[r] = segments with exactly r+1 tiles,
// counters[14] = most tiles of a segment (R).  Cleared by k_ds_prepare.
template <int UNUSED = 0>
__global__ void __launch_bounds__(BLOCK) k_ds_count(SegList sl, const u32* __restrict__ tile_start,
                                                    u32* __restrict__ more,
                                                    u32* __restrict__ counters) {
  const u32 n_seg = sl.n();
  u32 m = 0;
  for (u32 s = blockIdx.x * BLOCK + threadIdx.x; s < n_seg; s += gridDim.x * BLOCK) {
    const u32 nt = tile_start[s + 1] - tile_start[s];
    atomicAdd(&more[nt - 1], 1u);
    m = max(m, nt);
  }
  m = wave_max(m);
  if (__lane_id() == 0 && m) atomicMax(&counters[14], m);
}

// Step 2 (one workgroup of 1024 threads): more[r] = segments with more than
// r tiles (suffix sums), round0[r] = first claim index of round r (prefix
// sums of more), round0[R] = all tiles.
template <int UNUSED = 0>
__global__ void __launch_bounds__(1024) k_ds_rounds(const u32* __restrict__ counters,
                                                    u32* __restrict__ more,
                                                    u32* __restrict__ round0) {
  __shared__ u32 sm[17];
  const u32 tid = threadIdx.x;
  const u32 R = counters[14];
  const u32 chunk = (R + 1023) / 1024;
  {
    const u32 ct = 1023 - tid;  // chunks in reverse thread order: exclusive = later chunks
    const u32 lo = min(R, ct * chunk), hi = min(R, lo + chunk);
    u32 local = 0;
    for (u32 i = lo; i < hi; ++i) local += more[i];
    u32 tot;
    u32 acc = block_excl_sum<16>(local, sm, &tot);
    for (u32 i = hi; i > lo; --i) {
      acc += more[i - 1];
      more[i - 1] = acc;
    }
  }
  __syncthreads();
  {
    const u32 lo = min(R, tid * chunk), hi = min(R, lo + chunk);
    u32 local = 0;
    for (u32 i = lo; i < hi; ++i) local += more[i];
    u32 tot;
    u32 acc = block_excl_sum<16>(local, sm, &tot);
    for (u32 i = lo; i < hi; ++i) {
      round0[i] = acc;
      acc += more[i];
    }
    if (tid == 0) round0[R] = tot;
  }
}

// Position of every segment inside the rounds it takes part in: segments
// with more tiles first (ties in any order), so that the segments active in
// round r occupy positions [0, more[r]).  Also collects the passes any
// segment needs into counters[15].
template <int UNUSED = 0>
__global__ void __launch_bounds__(BLOCK) k_ds_pos(SegList sl, const u32* __restrict__ tile_start,
                                                  const u32* __restrict__ more,
                                                  u32* __restrict__ ties, u32* __restrict__ pos,
                                                  const u32* __restrict__ seg_mask,
                                                  u32* __restrict__ counters) {
  const u32 n_seg = sl.n();
  u32 need = 0;
  for (u32 s = blockIdx.x * BLOCK + threadIdx.x; s < n_seg; s += gridDim.x * BLOCK) {
    const u32 nt = tile_start[s + 1] - tile_start[s];
    pos[s] = more[nt] + atomicAdd(&ties[nt - 1], 1u);
    need |= seg_mask[s] & 0xFFu;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) need |= __shfl_xor(need, o, 64);
  if (__lane_id() == 0 && need) atomicOr(&counters[15], need);
}

// Descriptor of every tile at its claim index round0[t_in] + pos[seg].
template <int UNUSED = 0>
__global__ void __launch_bounds__(BLOCK) k_ds_desc(SegList sl, const u32* __restrict__ tile_start,
                                                   const u32* __restrict__ round0,
                                                   const u32* __restrict__ pos,
                                                   const u32* __restrict__ seg_mask,
                                                   TileDesc* __restrict__ desc) {
  const u32 n_seg = sl.n();
  const u32 total = tile_start[n_seg];
  for (u32 g = blockIdx.x * BLOCK + threadIdx.x; g < total; g += gridDim.x * BLOCK) {
    const u32 s = find_seg(tile_start, n_seg, g);
    const u32 t = g - tile_start[s];
    const u64 a = sl.lo[s], b = sl.hi[s];
    const u64 base = a + (u64)t * TILE;
    TileDesc d;
    d.base = base;
    d.seg = s;
    d.t_in = t;
    d.cnt = base < b ? (u32)min<u64>(TILE, b - base) : 0u;
    d.g = g;
    d.mask = seg_mask[s];
    d.pad = 0;
    desc[round0[t] + pos[s]] = d;
  }
}

// The same descriptor with every field in scalar registers (it is uniform
// over the workgroup).  Bases reach 2^32 - 1: both halves are taken unsigned.
__device__ __forceinline__ TileDesc uniform_desc(const TileDesc& d) {
  TileDesc u;
  u.base = ((u64)first_lane((u32)(d.base >> 32)) << 32) | (u64)first_lane((u32)d.base);
  u.seg = first_lane(d.seg);
  u.t_in = first_lane(d.t_in);
  u.cnt = first_lane(d.cnt);
  u.g = first_lane(d.g);
  u.mask = first_lane(d.mask);
  u.pad = 0;
  return u;
}

// Per-pass claim lists: a tile is sorted in pass p when its segment's digit
// p varies; pass 0 also takes the segments that need no pass and the
// unsupported ones (both are copied).
__device__ __forceinline__ bool in_pass(u32 mask, u32 p) {
  if (mask & SEG_UNSUPPORTED) return p == 0;
  return ((mask >> p) & 1u) || (p == 0 && mask == 0);
}

// Step 1: per block of LIST_BLK claims, how many are in each pass's list.
template <int PASSES>
__global__ void __launch_bounds__(LIST_BLK) k_ds_lcount(const u32* __restrict__ tile_start,
                                                        SegList sl,
                                                        const TileDesc* __restrict__ desc,
                                                        u32* __restrict__ lcount, u32 nblk) {
  const u32 total = tile_start[sl.n()];
  const u32 c = blockIdx.x * LIST_BLK + threadIdx.x;
  const bool have = c < total;  // claim slots past the last tile are in no list
  const u32 mask = have ? desc[c].mask : 0u;
#pragma unroll
  for (int p = 0; p < PASSES; ++p) {
    const int cnt = __syncthreads_count(have && in_pass(mask, p));
    if (threadIdx.x == 0) lcount[(u64)p * (nblk + 1) + blockIdx.x] = (u32)cnt;
  }
}

// Step 2 (one workgroup): block counts -> exclusive offsets per pass, and
// each list's size at index nblk.
template <int PASSES>
__global__ void __launch_bounds__(1024) k_ds_lscan(u32* __restrict__ lcount, u32 nblk) {
  __shared__ u32 sm[17];
  for (int p = 0; p < PASSES; ++p) {
    u32* lc = lcount + (u64)p * (nblk + 1);
    u32 carry = 0;
    for (u32 b0 = 0; b0 < nblk; b0 += 1024) {
      const u32 b = b0 + threadIdx.x;
      const u32 v = b < nblk ? lc[b] : 0u;
      u32 tot;
      const u32 ex = block_excl_sum<16>(v, sm, &tot);
      if (b < nblk) lc[b] = carry + ex;
      carry += tot;
    }
    if (threadIdx.x == 0) lc[nblk] = carry;
    __syncthreads();
  }
}

// Step 3: the lists, in claim order.
template <int PASSES>
__global__ void __launch_bounds__(LIST_BLK) k_ds_lfill(const u32* __restrict__ tile_start,
                                                       SegList sl,
                                                       const TileDesc* __restrict__ desc,
                                                       const u32* __restrict__ lcount, u32 nblk,
                                                       u32* __restrict__ lists, u64 max_tiles) {
  __shared__ u32 sm[17];
  const u32 total = tile_start[sl.n()];
  const u32 c = blockIdx.x * LIST_BLK + threadIdx.x;
  const bool have = c < total;  // claim slots past the last tile are in no list
  const u32 mask = have ? desc[c].mask : 0u;
#pragma unroll
  for (int p = 0; p < PASSES; ++p) {
    const bool in = have && in_pass(mask, p);
    u32 tot;
    const u32 ex = block_excl_sum<16>(in ? 1u : 0u, sm, &tot);
    if (in) lists[(u64)p * max_tiles + lcount[(u64)p * (nblk + 1) + blockIdx.x] + ex] = c;
  }
}

// In-place sorts: the tiles of segments with an odd number of active
// passes are copied to the tmp arrays, where their first pass reads them.
template <int UNUSED = 0>
__global__ void __launch_bounds__(BLOCK) k_ds_copy_odd(DigitSortBufs bf, SegList sl) {
  const u32 n_seg = sl.n();
  const u32 total = bf.tile_start[n_seg];
  for (u32 tile = blockIdx.x; tile < total; tile += gridDim.x) {
    u32 seg, t_in, cnt;
    u64 a, b, base;
    seg_tile_range(sl, bf.tile_start, n_seg, tile, seg, t_in, a, b, base, cnt);
    const u32 m = bf.seg_mask[seg];
    if (m == 0 || (m & SEG_UNSUPPORTED) || (__popc(m) & 1) == 0) continue;
    for (u32 i = threadIdx.x; i < cnt; i += BLOCK) {
      bf.keys_tmp[base + i] = bf.keys_out[base + i];
      bf.rids_tmp[base + i] = bf.rids_out[base + i];
      if (bf.vals_out) bf.vals_tmp[base + i] = bf.vals_out[base + i];
    }
  }
}

// Geometry of the scatter pass: PASS_WAVES waves per workgroup, so that two
// workgroups per CU keep 4*PASS_WAVES/4 waves on each SIMD while the tile stays
// TILE entries.
#ifndef KPA_PASS_WAVES
#define KPA_PASS_WAVES 8
#endif
constexpr int PASS_WAVES = KPA_PASS_WAVES;
constexpr int PASS_THREADS = PASS_WAVES * 64;
constexpr int PASS_ITEMS = TILE / PASS_THREADS;
static_assert(PASS_THREADS >= RADIX && PASS_ITEMS * PASS_THREADS == TILE, "pass geometry");

// One scatter pass over all tiles (persistent workgroups claiming tiles in
// the order of the tile descriptors).  A workgroup claims its next tile and
// issues that tile's loads as soon as the current one is staged in LDS, so
// that the loads are in flight during the current tile's look-back and
// write.  The prefetched tile publishes its counts only after the current
// one is written; every wait of a look-back still goes to a tile claimed
// earlier, so the waits cannot form a cycle.
//
// VALS: the value column moves with the keys: after a tile's keys and row
// ids are written, its values (loaded during the look-back) go through the
// key slots of LDS to the same destinations.
template <class DF, bool VALS>
__global__ void __launch_bounds__(PASS_THREADS, PASS_WAVES / 2)
    k_ds_pass(DigitSortBufs bf, SegList sl, typename DF::Params prm, u32 pass,
              u32* __restrict__ status_cur, u32* __restrict__ status_next) {
  __shared__ OnesweepSmemT<PASS_WAVES> sm;
  __shared__ float dfsm[DF::SMEM];
  const u32 tid = threadIdx.x;
  const u32 n_seg = sl.n();
  const u32 total = bf.tile_start[n_seg];
  const u32 nblk = (u32)list_blocks(bf.max_tiles);
  const u32* list = bf.order.lists + (u64)pass * bf.max_tiles;
  const u32 nlist = bf.order.lcount[(u64)pass * (nblk + 1) + nblk];
  const bool full = nlist == total;  // every tile takes part: list index = claim index
  // The next pass's look-back rows of the tiles it sorts start at zero (that
  // buffer is not used by this pass).
  if (pass + 1 < (u32)DF::PASSES) {
    const u32* nl = bf.order.lists + (u64)(pass + 1) * bf.max_tiles;
    const u32 nn = bf.order.lcount[(u64)(pass + 1) * (nblk + 1) + nblk];
    constexpr u32 ROWS = PASS_THREADS / RADIX;
    for (u32 r = blockIdx.x * ROWS + tid / RADIX; r < nn; r += gridDim.x * ROWS)
      status_next[(u64)bf.order.desc[nn == total ? r : nl[r]].g * RADIX + tid % RADIX] = 0;
  }
  u32* counter = bf.counters + pass;
  // Takes the next tile of this pass's list; false when none is left.  A
  // segment that needs no pass at all is copied in pass 0.
  auto claim = [&](TileDesc& td) -> bool {
    while (true) {
      __syncthreads();
      if (tid == 0) sm.tile = atomicAdd(counter, 1u);
      __syncthreads();
      const u32 k = first_lane(sm.tile);  // uniform: scalar loads below
      if (k >= nlist) return false;
      td = uniform_desc(bf.order.desc[full ? k : first_lane(list[k])]);
      if (td.mask == 0 || (td.mask & SEG_UNSUPPORTED)) {
        if (bf.keys_in != bf.keys_out) {
          for (u32 i = tid; i < td.cnt; i += PASS_THREADS) {
            bf.keys_out[td.base + i] = bf.keys_in[td.base + i];
            bf.rids_out[td.base + i] = bf.rids_in ? bf.rids_in[td.base + i] : (u32)(td.base + i);
            if (VALS) bf.vals_out[td.base + i] = bf.vals_in[td.base + i];
          }
        }
        continue;
      }
      return true;
    }
  };
  // Issues a claimed tile's loads (the pass's source buffer depends on how
  // many of the segment's passes came before); returns the present-item bits.
  auto load = [&](const TileDesc& td, u64 (&kk)[PASS_ITEMS], u32 (&rr)[PASS_ITEMS]) -> u32 {
    const u32 k = __popc(td.mask), q = __popc(td.mask & ((1u << pass) - 1));
    const bool from_in = q == 0 && !bf.in_place;
    const u64* src_k = from_in ? bf.keys_in : (((k - q) & 1) == 0 ? bf.keys_out : bf.keys_tmp);
    const u32* src_r = from_in ? bf.rids_in : (((k - q) & 1) == 0 ? bf.rids_out : bf.rids_tmp);
    u32 valid = 0;
#pragma unroll
    for (int j = 0; j < PASS_ITEMS; ++j) {
      const u32 o = tile_offset_t<PASS_WAVES>(j);
      if (o < td.cnt) {
        kk[j] = src_k[td.base + o];
        rr[j] = src_r ? src_r[td.base + o] : (u32)(td.base + o);  // no input rids: positions
        valid |= 1u << j;
      } else {
        kk[j] = 0;
        rr[j] = 0;
      }
    }
    return valid;
  };

  TileDesc td;
  if (!claim(td)) return;
  u64 kk[PASS_ITEMS];
  u32 rr[PASS_ITEMS];
  u32 valid = load(td, kk, rr);
  typename DF::Staged stg = DF::fetch(prm, td.seg);  // the digit function of the next segment
  u32 bound = 0xFFFFFFFFu;  // segment whose digit function is in dfsm
  DF df;
  while (true) {
    const u32 k = __popc(td.mask), q = __popc(td.mask & ((1u << pass) - 1));
    u64* dst_k = ((k - 1 - q) & 1) == 0 ? bf.keys_out : bf.keys_tmp;
    u32* dst_r = ((k - 1 - q) & 1) == 0 ? bf.rids_out : bf.rids_tmp;
    const u64 seg_start = td.base - (u64)td.t_in * TILE;
    const u64 my_base =
        tid < RADIX ? seg_start + bf.hist[((u64)td.seg * DF::PASSES + pass) * RADIX + tid] : 0ull;
    if (td.seg != bound) {
      // the previous tile's digits were computed before its barriers
      df = DF(stg);
      df.bind_staged(stg, dfsm);
      if (DF::SMEM > 1) __syncthreads();
      bound = td.seg;
    }
    u32 dd[PASS_ITEMS];
#pragma unroll
    for (int j = 0; j < PASS_ITEMS; ++j) dd[j] = ((valid >> j) & 1) ? df.digit(kk[j], pass) : 0u;
    u32 tile_count;
    u32 pos[PASS_ITEMS];
    const u32 cnt_d =
        VALS ? onesweep_rank_stage_pos(sm, kk, rr, dd, valid, status_cur, td.g, td.t_in,
                                       &tile_count, pos)
             : onesweep_rank_stage(sm, kk, rr, dd, valid, status_cur, td.g, td.t_in, &tile_count);
    // this tile's values, in flight during the look-back and the key write
    u64 vv[PASS_ITEMS];
    if (VALS) {
      const u64* src_v = (q == 0 && !bf.in_place)
                             ? bf.vals_in
                             : (((k - q) & 1) == 0 ? bf.vals_out : bf.vals_tmp);
#pragma unroll
      for (int j = 0; j < PASS_ITEMS; ++j) {
        const u32 o = tile_offset_t<PASS_WAVES>(j);
        vv[j] = ((valid >> j) & 1) ? src_v[td.base + o] : 0ull;
      }
    }
    const u32 cur_valid = valid;
    TileDesc nt;
    const bool more = claim(nt);
    const u32 nvalid = more ? load(nt, kk, rr) : 0u;
    if (more && nt.seg != td.seg) stg = DF::fetch(prm, nt.seg);  // in flight during the write
    onesweep_lookback_write(sm, status_cur, td.g, td.t_in, cnt_d, tile_count, my_base, dst_k,
                            dst_r);
    if (VALS) {
      u64* dst_v = ((k - 1 - q) & 1) == 0 ? bf.vals_out : bf.vals_tmp;
      write_staged_vals<OnesweepSmemT<PASS_WAVES>, PASS_WAVES, PASS_ITEMS>(sm, vv, pos, cur_valid,
                                                                          dst_v);
    }
    if (!more) return;
    td = nt;
    valid = nvalid;
  }
}

// Workgroups of `threads` threads that fit on the device at once for a kernel
// (persistent grids); computed once per kernel and thread count (kernels of
// one signature share a function-pointer type, so the cache is keyed by the
// kernel's address).
template <class K>
u32 resident_grid(K kernel, u32 cap, int threads = BLOCK) {
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, u32> cache;
  const std::pair<const void*, int> key{reinterpret_cast<const void*>(kernel), threads};
  u32 grid = 0;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) grid = it->second;
  }
  if (!grid) {
    int dev = 0, per_cu = 1;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return cap;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    grid = (u32)(p.multiProcessorCount * per_cu);
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = grid;
  }
  return grid < cap ? grid : cap;
}

// with_hist: count digits and derive offsets and pass masks here; otherwise
// the caller has filled b.hist (exclusive digit offsets per segment and pass)
// and b.seg_mask.
template <class DF>
kpa_status digit_sort_launch(const SegList& sl, const typename DF::Params& prm,
                             const DigitSortBufs& b, hipStream_t st, bool with_hist = true) {
  const bool radix = DF::PASSES == 8;
  KPA_CHECK(launch_seg_tiles_list(sl, TILE, b.tile_start, st));
  KPA_LAUNCH("sort_prepare", k_ds_prepare<0>, dim3(1024), dim3(BLOCK), 0, st, sl, b.tile_start,
             with_hist ? b.hist : nullptr, (u32)DF::PASSES, b.status0, b.counters, b.order,
             b.max_tiles);
  if (with_hist) {
    // tiles per workgroup: up to HIST_TILES_PER_BLOCK, fewer for small sorts
    // (a bundle's) so that they still spread over many workgroups
    const u32 tpb = (u32)std::min<u64>(HIST_TILES_PER_BLOCK,
                                       std::max<u64>(1, ceil_div(b.max_tiles, 2048)));
    const u32 hist_blocks = (u32)std::min<u64>(ceil_div(b.max_tiles, tpb), 4096);
    KPA_LAUNCH(radix ? "radix_hist" : "learned_hist", k_ds_hist<DF>, dim3(hist_blocks),
               dim3(BLOCK), 0, st, b.keys_in, sl, b.tile_start, prm, b.hist, tpb);
    KPA_LAUNCH(radix ? "radix_scan" : "learned_scan", k_ds_scan<DF>,
               dim3(std::min<u32>(sl.n_max, 2048)), dim3(BLOCK), 0, st, sl, b.hist, b.seg_mask,
               b.unsupported);
  }
  if (b.in_place)
    KPA_LAUNCH("sort_copy_odd", k_ds_copy_odd<0>,
               dim3((u32)std::min<u64>(std::max<u64>(b.max_tiles, 1), 4096)), dim3(BLOCK), 0, st,
               b, sl);
  const dim3 seg_grid((u32)std::min<u64>(ceil_div(std::max<u32>(sl.n_max, 1), BLOCK), 1024));
  KPA_LAUNCH("sort_count", k_ds_count<0>, seg_grid, dim3(BLOCK), 0, st, sl, b.tile_start,
             b.order.more, b.counters);
  KPA_LAUNCH("sort_rounds", k_ds_rounds<0>, dim3(1), dim3(1024), 0, st, b.counters, b.order.more,
             b.order.round0);
  KPA_LAUNCH("sort_order", k_ds_pos<0>, seg_grid, dim3(BLOCK), 0, st, sl, b.tile_start,
             b.order.more, b.order.ties, b.order.pos, b.seg_mask, b.counters);
  KPA_LAUNCH("sort_desc", k_ds_desc<0>,
             dim3((u32)std::min<u64>(ceil_div(b.max_tiles, BLOCK), 4096)), dim3(BLOCK), 0, st,
             sl, b.tile_start, b.order.round0, b.order.pos, b.seg_mask, b.order.desc);
  static_assert(DF::PASSES <= LIST_PASSES, "claim lists per pass");
  const u32 nblk = (u32)list_blocks(b.max_tiles);
  KPA_LAUNCH("sort_lists", k_ds_lcount<DF::PASSES>, dim3(nblk), dim3(LIST_BLK), 0, st,
             b.tile_start, sl, b.order.desc, b.order.lcount, nblk);
  KPA_LAUNCH("sort_lists", k_ds_lscan<DF::PASSES>, dim3(1), dim3(1024), 0, st, b.order.lcount,
             nblk);
  KPA_LAUNCH("sort_lists", k_ds_lfill<DF::PASSES>, dim3(nblk), dim3(LIST_BLK), 0, st,
             b.tile_start, sl, b.order.desc, b.order.lcount, nblk, b.order.lists, b.max_tiles);
  const bool vals = b.vals_in != nullptr;
  const u32 cap = (u32)std::min<u64>(b.max_tiles, 1u << 20);
  const u32 grid = vals ? resident_grid(k_ds_pass<DF, true>, cap, PASS_THREADS)
                        : resident_grid(k_ds_pass<DF, false>, cap, PASS_THREADS);
  const char* pname = radix ? "radix_pass" : (DF::PASSES == 2 ? "learned_scatter" : "pivot_scatter");
  for (u32 p = 0; p < (u32)DF::PASSES; ++p) {
    u32* cur = (p & 1) ? b.status1 : b.status0;
    u32* nxt = (p & 1) ? b.status0 : b.status1;
    if (vals)
      KPA_LAUNCH(pname, (k_ds_pass<DF, true>), dim3(grid), dim3(PASS_THREADS), 0, st, b, sl, prm,
                 p, cur, nxt);
    else
      KPA_LAUNCH(pname, (k_ds_pass<DF, false>), dim3(grid), dim3(PASS_THREADS), 0, st, b, sl, prm,
                 p, cur, nxt);
  }
  return KPA_OK;
}

}  // namespace kpa
