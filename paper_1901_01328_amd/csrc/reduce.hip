// Keyed reduction (Table 2; Sec. 4.2 keyed aggregation: scan a sorted KPA, follow the pointers
// and coalesce a nonresident column over each contiguous run of equal keys)
// and top-k groups by sum.
//
// Reduction over 4096-entry tiles of every segment:
//   1. heads: per tile, the number of runs that start in it (keys only);
//   2. scan (three short launches: sums of 1024-tile blocks, their prefix,
//      then each tile's): groups started before each tile; output slots of
//      runs that cross a tile edge are zeroed;
//   3. main: per tile, gather values, segmented scan in registers/LDS, write
//      each run at its last entry in the tile -- stored when the run lies in
//      the tile, added atomically when it crosses an edge.
// Integer addition and max are associative and commutative (sums modulo
// 2^64), so the result does not depend on how the work is split.
#include <mutex>

#include <type_traits>

#include "reduce_internal.hpp"

namespace kpa {

constexpr u32 GT = 4096;  // groups per top-k tile
constexpr int TOPK_MAX = 16;

__device__ __forceinline__ SegAgg shfl_up_agg(const SegAgg& a, int o) {
  SegAgg r;
  r.f = __shfl_up(a.f, o, 64);
  r.c = __shfl_up(a.c, o, 64);
  r.s = __shfl_up(a.s, o, 64);
  r.m = __shfl_up(a.m, o, 64);
  r.hp = __shfl_up(a.hp, o, 64);
  return r;
}

// Exclusive segmented scan over the block, with `carry_in` before thread 0.
template <int NW>
__device__ __forceinline__ SegAgg block_excl_segscan(SegAgg v, const SegAgg& carry_in,
                                                     SegAgg* sm) {
  const u32 lane = __lane_id(), w = threadIdx.x >> 6;
  SegAgg incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    SegAgg t = shfl_up_agg(incl, o);
    if (lane >= (u32)o) incl = seg_combine(t, incl);
  }
  SegAgg ex = shfl_up_agg(incl, 1);
  if (lane == 0) ex = seg_identity();
  if (lane == 63) sm[w] = incl;
  __syncthreads();
  SegAgg pre = carry_in;
  for (u32 i = 0; i < w; ++i) pre = seg_combine(pre, sm[i]);
  __syncthreads();
  return seg_combine(pre, ex);
}

__device__ __forceinline__ u64 block_sum_u64(u64 v, u64* sm) {
  v = wave_sum(v);
  const u32 w = threadIdx.x >> 6;
  if (__lane_id() == 0) sm[w] = v;
  __syncthreads();
  u64 r = 0;
  for (int i = 0; i < WAVES; ++i) r += sm[i];
  __syncthreads();
  return r;
}
__device__ __forceinline__ u64 block_max_u64(u64 v, u64* sm) {
  v = wave_max(v);
  const u32 w = threadIdx.x >> 6;
  if (__lane_id() == 0) sm[w] = v;
  __syncthreads();
  u64 r = 0;
  for (int i = 0; i < WAVES; ++i) r = sm[i] > r ? sm[i] : r;
  __syncthreads();
  return r;
}

struct TileRange {
  u32 seg;
  u64 a, b, base;
  u32 cnt;
};

__device__ __forceinline__ TileRange tile_range(const u64* seg_off, const u32* tile_start,
                                                const u32* tile_seg, u32 tile, u32 tsize) {
  TileRange r;
  r.seg = tile_seg[tile];
  r.a = seg_off[r.seg];
  r.b = seg_off[r.seg + 1];
  r.base = r.a + (u64)(tile - tile_start[r.seg]) * tsize;
  r.cnt = r.base < r.b ? (u32)min<u64>(tsize, r.b - r.base) : 0u;
  return r;
}

struct ValSrc {
  const unsigned char* rows;
  u32 row_bytes, val_off, val_w, on;
  __device__ __forceinline__ u64 operator()(u32 rid) const {
    return on ? load_val(rows, rid, row_bytes, val_off, val_w) : 0ull;
  }
};

// LDS index with one pad word per 16 entries, so that lanes reading
// consecutive-per-thread entries fall into different banks.
__device__ __forceinline__ u32 pidx(u32 i) { return i + (i >> 4); }
constexpr u32 PTILE = TILE + TILE / 16;

// Pass 1: runs that start in each tile; whether the tile's last run goes on
// into the next tile (flag bit 0).
__global__ void __launch_bounds__(BLOCK) k_reduce_heads(const u64* __restrict__ keys,
                                                        const u64* __restrict__ seg_off,
                                                        const u32* __restrict__ tile_start,
                                                        const u32* __restrict__ tile_seg,
                                                        u32 n_seg, u32* __restrict__ heads,
                                                        u32* __restrict__ flags) {
  __shared__ u64 sk[PTILE];
  __shared__ u64 red[WAVES];
  const u32 tile = blockIdx.x;
  if (tile >= tile_start[n_seg]) return;
  const TileRange tr = tile_range(seg_off, tile_start, tile_seg, tile, TILE);
  const u32 tid = threadIdx.x;
  {
    u64 kv[ITEMS];  // all loads of the thread in flight together
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const u32 i = tid + j * BLOCK;
      kv[j] = i < tr.cnt ? keys[tr.base + i] : 0ull;
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const u32 i = tid + j * BLOCK;
      if (i < tr.cnt) sk[pidx(i)] = kv[j];
    }
  }
  const bool has_prev = tr.base > tr.a;
  const u64 prev = has_prev ? keys[tr.base - 1] : 0ull;
  const bool has_next = tr.base + tr.cnt < tr.b;
  const u64 next = has_next ? keys[tr.base + tr.cnt] : 0ull;
  __syncthreads();
  u32 nh = 0;
  u64 before = tid == 0 ? prev : sk[pidx(tid * ITEMS - 1)];
  const bool first_has_prev = tid == 0 ? has_prev : true;
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const u32 idx = tid * ITEMS + j;
    if (idx < tr.cnt) {
      const u64 k = sk[pidx(idx)];
      const bool h = j == 0 ? (!first_has_prev || k != before) : (k != before);
      nh += h;
      before = k;
    }
  }
  const u64 total = block_sum_u64(nh, red);
  if (tid == 0) {
    heads[tile] = (u32)total;
    flags[tile] = (tr.cnt && has_next && sk[pidx(tr.cnt - 1)] == next) ? 1u : 0u;
  }
}

// Pass 2: groups started before each tile, in three launches over blocks of
// SCAN_TILES tiles: the heads of each block, the exclusive prefix of the block
// sums (and the total), then each tile's prefix.  Output slots of runs that
// cross a tile boundary are zeroed (those runs are accumulated with atomics
// in pass 3), and the first tile of each segment gives the segment's first
// group.
__global__ void __launch_bounds__(SCAN_TILES) k_reduce_bsum(const u32* __restrict__ heads,
                                                            const u32* __restrict__ tile_start,
                                                            u32 n_seg, u64* __restrict__ bsum) {
  __shared__ u64 red[SCAN_TILES / 64];
  const u32 n_tiles = tile_start[n_seg];
  const u32 t = blockIdx.x * SCAN_TILES + threadIdx.x;
  u64 v = wave_sum((u64)(t < n_tiles ? heads[t] : 0u));
  if (__lane_id() == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    u64 tot = 0;
    for (u32 i = 0; i < SCAN_TILES / 64; ++i) tot += red[i];
    bsum[blockIdx.x] = tot;
  }
}

// One workgroup: exclusive prefix of the nb block sums in place; the total
// is the number of groups (gseg_off[n_seg]).
__global__ void __launch_bounds__(1024) k_reduce_btop(u64* __restrict__ bsum, u32 nb, u32 n_seg,
                                                      u64* __restrict__ gseg_off) {
  __shared__ u64 wh[17];
  const u32 tid = threadIdx.x, lane = __lane_id(), w = tid >> 6;
  const u32 per = (nb + 1023) / 1024;
  const u32 b0 = min(nb, tid * per), b1 = min(nb, b0 + per);
  u64 H = 0;
  for (u32 b = b0; b < b1; ++b) H += bsum[b];
  u64 hi = H;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const u64 th = __shfl_up(hi, o, 64);
    if (lane >= (u32)o) hi += th;
  }
  if (lane == 63) wh[w] = hi;
  __syncthreads();
  u64 h = hi - H;
  for (u32 i = 0; i < w; ++i) h += wh[i];
  for (u32 b = b0; b < b1; ++b) {
    const u64 c = bsum[b];
    bsum[b] = h;
    h += c;
  }
  if (tid == 1023) gseg_off[n_seg] = h;
}

__global__ void __launch_bounds__(SCAN_TILES) k_reduce_bapply(
    const u32* __restrict__ heads, const u32* __restrict__ flags,
    const u32* __restrict__ tile_start, const u32* __restrict__ tile_seg, u32 n_seg,
    const u64* __restrict__ bpre, u64* __restrict__ gbase, u64* __restrict__ gseg_off,
    u64* __restrict__ o_cnt, u64* __restrict__ o_sum, u64* __restrict__ o_max) {
  __shared__ u32 sc[SCAN_TILES / 64 + 1];
  const u32 n_tiles = tile_start[n_seg];
  const u32 t = blockIdx.x * SCAN_TILES + threadIdx.x;
  const u32 hd = t < n_tiles ? heads[t] : 0u;
  u32 tot;
  const u32 ex = block_excl_sum<SCAN_TILES / 64>(hd, sc, &tot);
  if (t >= n_tiles) return;
  const u64 g0 = bpre[blockIdx.x] + ex;
  gbase[t] = g0;
  if (flags && (flags[t] & 1u)) {
    const u64 g = g0 + hd - 1;
    if (o_cnt) o_cnt[g] = 0;
    if (o_sum) o_sum[g] = 0;
    if (o_max) o_max[g] = 0;
  }
  const u32 s = tile_seg[t];
  if (tile_start[s] == t) gseg_off[s] = g0;
}

// Pass 3: gather values, segmented reduction of each tile in registers and
// LDS, write every run at its last entry in the tile.  A run wholly inside
// the tile is stored; a run crossing a tile edge adds its part atomically
// (integer sums and maxima are exact in any order).
__global__ void __launch_bounds__(BLOCK) k_reduce_main(
    const u64* __restrict__ keys, const u32* __restrict__ rids, const u64* __restrict__ seg_off,
    const u32* __restrict__ tile_start, const u32* __restrict__ tile_seg, u32 n_seg, ValSrc vs,
    const u64* __restrict__ gbase,
    u64* __restrict__ o_key, u64* __restrict__ o_cnt, u64* __restrict__ o_sum,
    u64* __restrict__ o_max, u64* __restrict__ o_start) {
  __shared__ u64 sk[PTILE];
  __shared__ u32 sr[PTILE];
  __shared__ SegAgg wsm[WAVES];
  __shared__ u32 hsm[WAVES + 1];
  const u32 tile = blockIdx.x;
  if (tile >= tile_start[n_seg]) return;
  const TileRange tr = tile_range(seg_off, tile_start, tile_seg, tile, TILE);
  const u32 tid = threadIdx.x;
  {
    u64 kv[ITEMS];  // all loads of the thread in flight together
    u32 rv[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const u32 i = tid + j * BLOCK;
      kv[j] = i < tr.cnt ? keys[tr.base + i] : 0ull;
      // without row ids, entry i's row is row i (values already in KPA order)
      rv[j] = i < tr.cnt ? (rids ? rids[tr.base + i] : (u32)(tr.base + i)) : 0u;
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const u32 i = tid + j * BLOCK;
      if (i < tr.cnt) {
        sk[pidx(i)] = kv[j];
        sr[pidx(i)] = rv[j];
      }
    }
  }
  const bool has_prev = tr.base > tr.a;
  const u64 prev = has_prev ? keys[tr.base - 1] : 0ull;
  const bool has_next = tr.base + tr.cnt < tr.b;
  const u64 next = has_next ? keys[tr.base + tr.cnt] : 0ull;
  __syncthreads();

  u64 v[ITEMS];
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const u32 idx = tid * ITEMS + j;
    v[j] = idx < tr.cnt ? vs(sr[pidx(idx)]) : 0ull;
  }
  u32 hmask = 0, tmask = 0;
  u64 before = tid == 0 ? prev : (tid * ITEMS - 1 < tr.cnt ? sk[pidx(tid * ITEMS - 1)] : 0ull);
  const bool lead_has_prev = tid == 0 ? has_prev : true;
  u64 kr[ITEMS];  // the thread's keys (sk is reused for the outputs below)
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const u32 idx = tid * ITEMS + j;
    kr[j] = 0ull;
    if (idx < tr.cnt) {
      const u64 k = sk[pidx(idx)];
      kr[j] = k;
      const bool h = j == 0 ? (!lead_has_prev || k != before) : (k != before);
      const bool last = idx + 1 == tr.cnt;
      const u64 after = last ? next : sk[pidx(idx + 1)];
      const bool t = last ? (!has_next || k != after) : (k != after);
      hmask |= (u32)h << j;
      tmask |= (u32)t << j;
      before = k;
    }
  }
  SegAgg A = seg_identity();
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const u32 idx = tid * ITEMS + j;
    if (idx < tr.cnt) A = seg_combine(A, SegAgg{(hmask >> j) & 1u, 1ull, v[j], v[j], tr.base + idx});
  }
  u32 htot;
  const u32 hex = block_excl_sum((u32)__popc(hmask), hsm, &htot);
  SegAgg run = block_excl_segscan<WAVES>(A, seg_identity(), wsm);
  const u64 gb = gbase[tile];
  // Group columns gathered in LDS one at a time and written contiguously (as
  // in k_reduce_main_seq); sk is free: the scans above end with barriers.
  const bool last_goes_on = has_next && tr.cnt && keys[tr.base + tr.cnt - 1] == next;
  const u32 nfull = htot - (last_goes_on && htot ? 1u : 0u);
  const SegAgg run0 = run;
  auto column = [&](auto fc, u64* __restrict__ out) {
    constexpr int F = decltype(fc)::value;
    SegAgg r = run0;
    u32 hs = hex;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const u32 idx = tid * ITEMS + j;
      if (idx < tr.cnt) {
        const u32 h = (hmask >> j) & 1u;
        r = seg_combine(r, SegAgg{h, 1ull, v[j], v[j], tr.base + idx});
        hs += h;
        const bool t = (tmask >> j) & 1u;
        const bool cont = idx + 1 == tr.cnt && !t;  // the run goes on in the next tile
        if (t || cont) {
          if (r.f) sk[hs - 1] = F == 0 ? kr[j] : F == 1 ? r.c : F == 2 ? r.s : F == 3 ? r.m : r.hp;
          if (F == 0 && !(r.f && t)) {
            const u64 gi = gb + hs - 1;
            if (o_cnt) atomicAdd(reinterpret_cast<unsigned long long*>(o_cnt + gi), r.c);
            if (o_sum) atomicAdd(reinterpret_cast<unsigned long long*>(o_sum + gi), r.s);
            if (o_max) atomicMax(reinterpret_cast<unsigned long long*>(o_max + gi), r.m);
          }
        }
      }
    }
    __syncthreads();
    const u32 lim = (F == 0 || F == 4) ? htot : nfull;
    for (u32 i = tid; i < lim; i += BLOCK) out[gb + i] = sk[i];
    __syncthreads();
  };
  column(std::integral_constant<int, 0>(), o_key);
  if (o_cnt) column(std::integral_constant<int, 1>(), o_cnt);
  if (o_sum) column(std::integral_constant<int, 2>(), o_sum);
  if (o_max) column(std::integral_constant<int, 3>(), o_max);
  if (o_start) column(std::integral_constant<int, 4>(), o_start);
}

// ---- pass 3 when the values are already in KPA order (8-byte values, row
// ids NULL): no gather; keys and values are loaded coalesced and staged one
// after the other through the same LDS tile (so four workgroups fit a CU),
// and the segmented scan across the wave runs on DPP lane moves.

// Aggregate of a partial run inside one tile (a tile holds at most 4096
// entries, so the count fits 32 bits); hp only when group starts are wanted.
template <bool START>
struct RunAgg {
  u32 f, c;
  u64 s, m;
  u64 hp;
};

template <bool START>
__device__ __forceinline__ RunAgg<START> run_combine(const RunAgg<START>& a,
                                                     const RunAgg<START>& b) {
  if (b.f) return b;
  RunAgg<START> r;
  r.f = a.f;
  r.c = a.c + b.c;
  r.s = a.s + b.s;
  r.m = a.m > b.m ? a.m : b.m;
  r.hp = START ? a.hp : 0ull;
  return r;
}

// The aggregate of the lane that the DPP control selects (identity where none).
template <int CTRL, int ROW_MASK, bool START>
__device__ __forceinline__ RunAgg<START> dpp_agg(const RunAgg<START>& a) {
  RunAgg<START> r;
  r.f = dpp32<CTRL, ROW_MASK>(0u, a.f);
  r.c = dpp32<CTRL, ROW_MASK>(0u, a.c);
  r.s = dpp64<CTRL, ROW_MASK>(0ull, a.s);
  r.m = dpp64<CTRL, ROW_MASK>(0ull, a.m);
  r.hp = START ? dpp64<CTRL, ROW_MASK>(0ull, a.hp) : 0ull;
  return r;
}

// Inclusive segmented scan over the wave (Hillis-Steele within rows of 16,
// then the two row broadcasts); the identity (all zero) fills lanes without
// a source, and run_combine(identity, x) == x.
template <bool START>
__device__ __forceinline__ RunAgg<START> wave_incl_runscan(RunAgg<START> x) {
  x = run_combine(dpp_agg<DPP_ROW_SHR + 1, 0xF>(x), x);
  x = run_combine(dpp_agg<DPP_ROW_SHR + 2, 0xF>(x), x);
  x = run_combine(dpp_agg<DPP_ROW_SHR + 4, 0xF>(x), x);
  x = run_combine(dpp_agg<DPP_ROW_SHR + 8, 0xF>(x), x);
  x = run_combine(dpp_agg<DPP_BCAST15, 0xA>(x), x);
  x = run_combine(dpp_agg<DPP_BCAST31, 0xC>(x), x);
  return x;
}

template <bool START>
__global__ void __launch_bounds__(BLOCK, 4) k_reduce_main_seq(
    const u64* __restrict__ keys, const u64* __restrict__ vals, const u64* __restrict__ seg_off,
    const u32* __restrict__ tile_start, const u32* __restrict__ tile_seg, u32 n_seg,
    const u64* __restrict__ gbase, u64* __restrict__ o_key, u64* __restrict__ o_cnt,
    u64* __restrict__ o_sum, u64* __restrict__ o_max, u64* __restrict__ o_start) {
  __shared__ u64 st[PTILE];  // the tile's keys, then its values
  __shared__ RunAgg<START> wsm[WAVES];
  __shared__ u32 hsm[WAVES + 1];
  const u32 tile = blockIdx.x;
  if (tile >= tile_start[n_seg]) return;
  const TileRange tr = tile_range(seg_off, tile_start, tile_seg, tile, TILE);
  const u32 tid = threadIdx.x;
  u64 k[ITEMS], v[ITEMS];
  u64 before, after;
  {
    u64 kv[ITEMS], vv[ITEMS];  // all loads of the thread in flight together
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const u32 i = tid + j * BLOCK;
      kv[j] = i < tr.cnt ? keys[tr.base + i] : 0ull;
      vv[j] = vals && i < tr.cnt ? vals[tr.base + i] : 0ull;
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const u32 i = tid + j * BLOCK;
      if (i < tr.cnt) st[pidx(i)] = kv[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const u32 idx = tid * ITEMS + j;
      k[j] = idx < tr.cnt ? st[pidx(idx)] : 0ull;
    }
    const u32 last = tid * ITEMS + ITEMS;  // the next thread's first entry
    before = tid > 0 && tid * ITEMS - 1 < tr.cnt ? st[pidx(tid * ITEMS - 1)] : 0ull;
    after = last < tr.cnt ? st[pidx(last)] : 0ull;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) v[j] = 0ull;
    if (vals) {  // uniform: without values (runs only) the second staging round is skipped
      __syncthreads();
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) {
        const u32 i = tid + j * BLOCK;
        if (i < tr.cnt) st[pidx(i)] = vv[j];
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) {
        const u32 idx = tid * ITEMS + j;
        v[j] = idx < tr.cnt ? st[pidx(idx)] : 0ull;
      }
    }
  }
  const bool has_prev = tr.base > tr.a;
  const bool has_next = tr.base + tr.cnt < tr.b;
  if (tid == 0) before = has_prev ? keys[tr.base - 1] : 0ull;
  const u64 next = has_next ? keys[tr.base + tr.cnt] : 0ull;
  const bool lead_has_prev = tid == 0 ? has_prev : true;
  u32 hmask = 0, tmask = 0;
  u64 prevk = before;
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const u32 idx = tid * ITEMS + j;
    if (idx < tr.cnt) {
      const bool h = j == 0 ? (!lead_has_prev || k[j] != prevk) : (k[j] != prevk);
      const bool lastent = idx + 1 == tr.cnt;
      const u64 nk = j + 1 < ITEMS ? k[j + 1] : after;
      const bool t = lastent ? (!has_next || k[j] != next) : (k[j] != nk);
      hmask |= (u32)h << j;
      tmask |= (u32)t << j;
      prevk = k[j];
    }
  }
  // this thread's aggregate, then the exclusive scan over the block
  RunAgg<START> A{0u, 0u, 0ull, 0ull, 0ull};
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const u32 idx = tid * ITEMS + j;
    if (idx < tr.cnt)
      A = run_combine(A, RunAgg<START>{(hmask >> j) & 1u, 1u, v[j], v[j], tr.base + idx});
  }
  u32 htot;
  const u32 hex = block_excl_sum((u32)__popc(hmask), hsm, &htot);
  const RunAgg<START> incl = wave_incl_runscan(A);
  const u32 lane = __lane_id(), w = tid >> 6;
  RunAgg<START> ex = dpp_agg<DPP_WAVE_SHR1, 0xF>(incl);
  if (lane == 0) ex = RunAgg<START>{0u, 0u, 0ull, 0ull, 0ull};
  if (lane == 63) wsm[w] = incl;
  __syncthreads();
  RunAgg<START> run{0u, 0u, 0ull, 0ull, 0ull};
  for (u32 i = 0; i < w; ++i) run = run_combine(run, wsm[i]);
  run = run_combine(run, ex);
  const u64 gb = gbase[tile];
  // The groups that start in the tile are gb + [0, htot).  Their columns are
  // gathered in LDS one at a time (st is free again: every thread has read
  // its entries before the barriers above), each by a walk over the thread's
  // entries, and written out contiguously: stores of single 8-byte words
  // from the lanes that end runs reach memory as separate partial writes.
  // A run that goes on into the next tile holds the tile's last group; its
  // count, sum and maximum are accumulated with atomics (here and in the
  // next tiles) onto the zeros the scan pass left there, as are those of a
  // run that began in an earlier tile.
  const bool last_goes_on = has_next && tr.cnt && keys[tr.base + tr.cnt - 1] == next;
  const u32 nfull = htot - (last_goes_on && htot ? 1u : 0u);
  const RunAgg<START> run0 = run;
  // column F (0 key, 1 count, 2 sum, 3 max, 4 start) into `out`; the walk of
  // column 0 also issues the atomics, and the keys are dead after it
  auto column = [&](auto fc, u64* __restrict__ out) {
    constexpr int F = decltype(fc)::value;
    RunAgg<START> r = run0;
    u32 hs = hex;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const u32 idx = tid * ITEMS + j;
      if (idx < tr.cnt) {
        const u32 h = (hmask >> j) & 1u;
        r = run_combine(r, RunAgg<START>{h, 1u, v[j], v[j], tr.base + idx});
        hs += h;
        const bool t = (tmask >> j) & 1u;
        const bool cont = idx + 1 == tr.cnt && !t;  // the run goes on in the next tile
        if (t || cont) {
          if (r.f)
            st[hs - 1] = F == 0 ? k[j] : F == 1 ? (u64)r.c : F == 2 ? r.s : F == 3 ? r.m : r.hp;
          if (F == 0 && !(r.f && t)) {
            const u64 gi = gb + hs - 1;
            if (o_cnt) atomicAdd(reinterpret_cast<unsigned long long*>(o_cnt + gi), (u64)r.c);
            if (o_sum) atomicAdd(reinterpret_cast<unsigned long long*>(o_sum + gi), r.s);
            if (o_max) atomicMax(reinterpret_cast<unsigned long long*>(o_max + gi), r.m);
          }
        }
      }
    }
    __syncthreads();
    const u32 lim = (F == 0 || F == 4) ? htot : nfull;
    for (u32 i = tid; i < lim; i += BLOCK) out[gb + i] = st[i];
    __syncthreads();
  };
  column(std::integral_constant<int, 0>(), o_key);
  if (o_cnt) column(std::integral_constant<int, 1>(), o_cnt);
  if (o_sum) column(std::integral_constant<int, 2>(), o_sum);
  if (o_max) column(std::integral_constant<int, 3>(), o_max);
  if (START) column(std::integral_constant<int, 4>(), o_start);
}

kpa_status launch_tile_scan(const u32* counts, const u32* tile_start, const u32* tile_seg,
                            u32 n_seg, u64 max_tiles, u64* bsum, u64* tbase, u64* seg_first,
                            hipStream_t st) {
  const u32 nb = (u32)ceil_div(max_tiles, SCAN_TILES);
  KPA_LAUNCH("tile_scan", k_reduce_bsum, dim3(nb), dim3(SCAN_TILES), 0, st, counts, tile_start,
             n_seg, bsum);
  KPA_LAUNCH("tile_scan", k_reduce_btop, dim3(1), dim3(1024), 0, st, bsum, nb, n_seg, seg_first);
  KPA_LAUNCH("tile_scan", k_reduce_bapply, dim3(nb), dim3(SCAN_TILES), 0, st, counts, nullptr,
             tile_start, tile_seg, n_seg, bsum, tbase, seg_first, nullptr, nullptr, nullptr);
  return KPA_OK;
}

void reduce_plan(u64 n_cap, u32 n_seg, Carver& c, ReduceWs* w) {
  w->max_tiles = max_tiles(n_cap, n_seg, TILE);
  w->tile_start = c.take<u32>((u64)n_seg + 1);
  w->tile_seg = c.take<u32>(w->max_tiles);
  w->heads = c.take<u32>(w->max_tiles);
  w->flags = c.take<u32>(w->max_tiles);
  w->gbase = c.take<u64>(w->max_tiles);
  w->bsum = c.take<u64>(ceil_div(w->max_tiles, SCAN_TILES));
}

kpa_status reduce_launch(const u64* keys, const u32* rids, const u64* seg_off, u32 n_seg,
                         const unsigned char* rows, const kpa_row_layout* L, bool need_val,
                         const ReduceOut& o, const ReduceWs& w, hipStream_t st) {
  ValSrc vs;
  vs.rows = rows;
  vs.row_bytes = L ? L->row_bytes : 0;
  vs.val_off = L ? L->val_off : 0;
  vs.val_w = L ? L->val_w : 8;
  vs.on = need_val ? 1u : 0u;
  KPA_CHECK(launch_seg_tiles(seg_off, nullptr, n_seg, TILE, w.tile_start, st));
  KPA_CHECK(launch_tile_seg(w.tile_start, n_seg, nullptr, w.max_tiles, w.tile_seg, st));
  KPA_LAUNCH("reduce_heads", k_reduce_heads, dim3((u32)w.max_tiles), dim3(BLOCK), 0, st, keys,
             seg_off, w.tile_start, w.tile_seg, n_seg, w.heads, w.flags);
  const u32 nb = (u32)ceil_div(w.max_tiles, SCAN_TILES);
  KPA_LAUNCH("reduce_scan", k_reduce_bsum, dim3(nb), dim3(SCAN_TILES), 0, st, w.heads,
             w.tile_start, n_seg, w.bsum);
  KPA_LAUNCH("reduce_scan", k_reduce_btop, dim3(1), dim3(1024), 0, st, w.bsum, nb, n_seg,
             o.gseg_off);
  KPA_LAUNCH("reduce_scan", k_reduce_bapply, dim3(nb), dim3(SCAN_TILES), 0, st, w.heads, w.flags,
             w.tile_start, w.tile_seg, n_seg, w.bsum, w.gbase, o.gseg_off, o.cnt, o.sum, o.max);
  // In KPA order (8-byte values, no row ids), or no values at all (runs,
  // counts and group starts only): the sequential kernel, which reads no
  // row ids; values are read through the row ids otherwise.
  const bool in_order = !rids && need_val && L && L->row_bytes == 8 && L->val_off == 0 &&
                        L->val_w == 8;
  const bool seq = in_order || !need_val;
  const u64* seq_vals = in_order ? reinterpret_cast<const u64*>(rows) : nullptr;
  if (seq && o.gstart)
    KPA_LAUNCH("reduce_main", k_reduce_main_seq<true>, dim3((u32)w.max_tiles), dim3(BLOCK), 0, st,
               keys, seq_vals, seg_off, w.tile_start, w.tile_seg, n_seg, w.gbase, o.gkey, o.cnt,
               o.sum, o.max, o.gstart);
  else if (seq)
    KPA_LAUNCH("reduce_main", k_reduce_main_seq<false>, dim3((u32)w.max_tiles), dim3(BLOCK), 0,
               st, keys, seq_vals, seg_off, w.tile_start, w.tile_seg, n_seg, w.gbase, o.gkey,
               o.cnt, o.sum, o.max, o.gstart);
  else
    KPA_LAUNCH("reduce_main", k_reduce_main, dim3((u32)w.max_tiles), dim3(BLOCK), 0, st, keys,
               rids, seg_off, w.tile_start, w.tile_seg, n_seg, vs, w.gbase, o.gkey, o.cnt, o.sum,
               o.max, o.gstart);
  return KPA_OK;
}

// ------------------------------------------------------------------ top-k --

// (sum desc, key asc) is a total order on groups of one segment.
__device__ __forceinline__ bool better(u64 sa, u64 ka, u64 sb, u64 kb) {
  return sa > sb || (sa == sb && ka < kb);
}

struct TopList {
  u64 s[TOPK_MAX], k[TOPK_MAX];
  u32 n;
  __device__ __forceinline__ void init() { n = 0; }
  // Keeps the best TOPK_MAX entries seen (a superset of the best k <= TOPK_MAX).
  __device__ __forceinline__ void insert(u64 xs, u64 xk) {
    if (n == TOPK_MAX && !better(xs, xk, s[TOPK_MAX - 1], k[TOPK_MAX - 1])) return;
#pragma unroll
    for (int j = 0; j < TOPK_MAX; ++j) {
      if ((u32)j < n) {
        if (better(xs, xk, s[j], k[j])) {
          u64 ts = s[j], tk = k[j];
          s[j] = xs;
          k[j] = xk;
          xs = ts;
          xk = tk;
        }
      } else if ((u32)j == n) {
        s[j] = xs;
        k[j] = xk;
      }
    }
    if (n < TOPK_MAX) ++n;
  }
  __device__ __forceinline__ void pop() {
#pragma unroll
    for (int j = 0; j + 1 < TOPK_MAX; ++j) {
      s[j] = s[j + 1];
      k[j] = k[j + 1];
    }
    --n;
  }
};

// Block-wide: emit the best `cap` entries of all threads' lists in order.
__device__ __forceinline__ u32 pop_merge(TopList& L, u32 cap, u64* out_s, u64* out_k, u64* sm_s,
                                         u64* sm_k, u32* sm_t) {
  const u32 tid = threadIdx.x, w = tid >> 6, lane = __lane_id();
  u32 got = 0;
  for (u32 r = 0; r < cap; ++r) {
    u32 has = L.n > 0;
    u64 bs = has ? L.s[0] : 0, bk = has ? L.k[0] : 0;
    u32 bt = tid;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      u32 oh = __shfl_xor(has, o, 64);
      u64 os = __shfl_xor(bs, o, 64), ok = __shfl_xor(bk, o, 64);
      u32 ot = __shfl_xor(bt, o, 64);
      bool take = oh && (!has || better(os, ok, bs, bk));
      if (take) {
        has = 1;
        bs = os;
        bk = ok;
        bt = ot;
      }
    }
    if (lane == 0) {
      sm_s[w] = bs;
      sm_k[w] = bk;
      sm_t[w] = has ? bt : 0xFFFFFFFFu;
    }
    __syncthreads();
    if (tid == 0) {
      u32 win = 0xFFFFFFFFu;
      u64 ws = 0, wk = 0;
      for (int i = 0; i < WAVES; ++i) {
        if (sm_t[i] == 0xFFFFFFFFu) continue;
        if (win == 0xFFFFFFFFu || better(sm_s[i], sm_k[i], ws, wk)) {
          win = sm_t[i];
          ws = sm_s[i];
          wk = sm_k[i];
        }
      }
      sm_t[WAVES] = win;
      if (win != 0xFFFFFFFFu) {
        out_s[r] = ws;
        out_k[r] = wk;
      }
    }
    __syncthreads();
    const u32 win = sm_t[WAVES];
    __syncthreads();
    if (win == 0xFFFFFFFFu) break;
    if (win == tid) L.pop();
    ++got;
  }
  return got;
}

__global__ void __launch_bounds__(BLOCK) k_topk_local(const u64* __restrict__ gkey,
                                                      const u64* __restrict__ gsum,
                                                      const u64* __restrict__ gseg_off,
                                                      const u32* __restrict__ tile_start,
                                                      const u32* __restrict__ tile_seg,
                                                      u32 n_seg, u32 k, u64* __restrict__ cs,
                                                      u64* __restrict__ ck,
                                                      u32* __restrict__ cn) {
  __shared__ u64 ss[WAVES], sk2[WAVES];
  __shared__ u32 st[WAVES + 1];
  __shared__ u64 os[TOPK_MAX], ok[TOPK_MAX];
  const u32 tile = blockIdx.x;
  if (tile >= tile_start[n_seg]) return;
  const TileRange tr = tile_range(gseg_off, tile_start, tile_seg, tile, GT);
  TopList L;
  L.init();
  for (u32 i = threadIdx.x; i < tr.cnt; i += BLOCK) L.insert(gsum[tr.base + i], gkey[tr.base + i]);
  const u32 got = pop_merge(L, k, os, ok, ss, sk2, st);
  if (threadIdx.x < got) {
    cs[(u64)tile * TOPK_MAX + threadIdx.x] = os[threadIdx.x];
    ck[(u64)tile * TOPK_MAX + threadIdx.x] = ok[threadIdx.x];
  }
  if (threadIdx.x == 0) cn[tile] = got;
}

__global__ void __launch_bounds__(BLOCK) k_topk_final(const u64* __restrict__ cs,
                                                      const u64* __restrict__ ck,
                                                      const u32* __restrict__ cn,
                                                      const u32* __restrict__ tile_start, u32 k,
                                                      u64* __restrict__ out_key,
                                                      u64* __restrict__ out_sum,
                                                      u32* __restrict__ out_n) {
  __shared__ u64 ss[WAVES], sk2[WAVES];
  __shared__ u32 st[WAVES + 1];
  __shared__ u64 os[TOPK_MAX], ok[TOPK_MAX];
  const u32 s = blockIdx.x;
  const u32 t0 = tile_start[s], t1 = tile_start[s + 1];
  TopList L;
  L.init();
  const u64 total = (u64)(t1 - t0) * TOPK_MAX;
  for (u64 i = threadIdx.x; i < total; i += BLOCK) {
    const u32 t = t0 + (u32)(i / TOPK_MAX);
    const u32 r = (u32)(i % TOPK_MAX);
    if (r < cn[t]) L.insert(cs[(u64)t * TOPK_MAX + r], ck[(u64)t * TOPK_MAX + r]);
  }
  const u32 got = pop_merge(L, k, os, ok, ss, sk2, st);
  if (threadIdx.x < got) {
    out_key[(u64)s * k + threadIdx.x] = ok[threadIdx.x];
    out_sum[(u64)s * k + threadIdx.x] = os[threadIdx.x];
  }
  if (threadIdx.x == 0) out_n[s] = got;
}

struct TopkWs {
  u32* tile_start;
  u32* tile_seg;
  u64* cs;
  u64* ck;
  u32* cn;
  u64 max_tiles;
};

static void topk_plan(u64 g_cap, u32 n_seg, Carver& c, TopkWs* w) {
  w->max_tiles = max_tiles(g_cap, n_seg, GT);
  w->tile_start = c.take<u32>((u64)n_seg + 1);
  w->tile_seg = c.take<u32>(w->max_tiles);
  w->cs = c.take<u64>(w->max_tiles * TOPK_MAX);
  w->ck = c.take<u64>(w->max_tiles * TOPK_MAX);
  w->cn = c.take<u32>(w->max_tiles);
}

}  // namespace kpa

using namespace kpa;

extern "C" {

kpa_status kpa_reduce_by_key_workspace_size(uint64_t n_cap, uint32_t n_seg, size_t* bytes) {
  clear_error();
  KPA_REQUIRE(bytes, KPA_EINVAL, "bytes is null");
  Carver c(nullptr);
  ReduceWs w;
  reduce_plan(n_cap, n_seg ? n_seg : 1, c, &w);
  *bytes = c.used + 256;
  return KPA_OK;
}

kpa_status kpa_reduce_by_key(const uint64_t* keys, const uint32_t* rids, const uint64_t* seg_off,
                             uint32_t n_seg, uint64_t n_cap, const void* rows,
                             const kpa_row_layout* layout, uint64_t* out_gkey, uint64_t* out_cnt,
                             uint64_t* out_sum, uint64_t* out_max, uint64_t* out_gstart,
                             uint64_t* out_gseg_off, void* ws, size_t ws_bytes,
                             hipStream_t stream) {
  clear_error();
  const bool need_val = out_sum || out_max;
  if (need_val) KPA_CHECK(check_layout(layout, true, false));
  if (n_seg == 0) return KPA_OK;
  KPA_REQUIRE(keys && seg_off && out_gkey && out_gseg_off && ws, KPA_EINVAL, "null pointer");
  KPA_REQUIRE(!need_val || rows, KPA_EINVAL, "rows needed for sum/max");
  KPA_REQUIRE(aligned(keys, 8) && aligned(rids, 4) && aligned(seg_off, 8) &&
                  aligned(out_gkey, 8) && aligned(out_gseg_off, 8) && aligned(ws, 256) &&
                  (!rows || aligned(rows, 16)),
              KPA_EINVAL, "misaligned pointer");
  KPA_REQUIRE(n_cap < (1ull << 32), KPA_EUNSUPPORTED, "n_cap must be below 2^32");
  Carver c(ws);
  ReduceWs w;
  reduce_plan(n_cap, n_seg, c, &w);
  KPA_REQUIRE(c.used <= ws_bytes, KPA_EWORKSPACE, "workspace too small: need %zu bytes", c.used);
  ReduceOut o{out_gkey, out_cnt, out_sum, out_max, out_gstart, out_gseg_off};
  return reduce_launch(keys, rids, seg_off, n_seg, static_cast<const unsigned char*>(rows),
                       layout, need_val, o, w, stream);
}

}  // extern "C"

// ------------------------------------------------------ no-allocation form --
// The reduction's tile bookkeeping (tile map, run-head counts, group bases,
// scan blocks) in a file-scope device array instead of a caller workspace.
// Each device holds its own copy; its address is looked up once per device
// and kept, and only that address is passed to kernels.

namespace kpa {
namespace {

constexpr size_t REDUCE_SCRATCH_BYTES = 4u << 20;
static __device__ __align__(256) unsigned char scratch[REDUCE_SCRATCH_BYTES];

constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

// The current device's copy of the array (looked up on the device's first use).
kpa_status scratch_ptr(void** out) {
  int dev = 0;
  KPA_HIP(hipGetDevice(&dev));
  KPA_REQUIRE(dev >= 0 && dev < SCRATCH_MAX_DEVICES, KPA_EUNSUPPORTED,
              "device index %d above %d", dev, SCRATCH_MAX_DEVICES - 1);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    KPA_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    KPA_REQUIRE(p != nullptr, KPA_EHIP, "no device address for the reduction's scratch array");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return KPA_OK;
}

}  // namespace
}  // namespace kpa

extern "C" {

kpa_status kpa_reduce_by_key_noalloc(const uint64_t* keys, const uint32_t* rids,
                                     const uint64_t* seg_off, uint32_t n_seg, uint64_t n_cap,
                                     const void* rows, const kpa_row_layout* layout,
                                     uint64_t* out_gkey, uint64_t* out_cnt, uint64_t* out_sum,
                                     uint64_t* out_max, uint64_t* out_gstart,
                                     uint64_t* out_gseg_off, hipStream_t stream) {
  clear_error();
  const bool need_val = out_sum || out_max;
  if (need_val) KPA_CHECK(check_layout(layout, true, false));
  if (n_seg == 0) return KPA_OK;
  KPA_REQUIRE(keys && seg_off && out_gkey && out_gseg_off, KPA_EINVAL, "null pointer");
  KPA_REQUIRE(!need_val || rows, KPA_EINVAL, "rows needed for sum/max");
  KPA_REQUIRE(aligned(keys, 8) && aligned(rids, 4) && aligned(seg_off, 8) &&
                  aligned(out_gkey, 8) && aligned(out_gseg_off, 8) && (!rows || aligned(rows, 16)),
              KPA_EINVAL, "misaligned pointer");
  KPA_REQUIRE(n_cap < (1ull << 32), KPA_EUNSUPPORTED, "n_cap must be below 2^32");
  KPA_REQUIRE(!prof_enabled(), KPA_EINVAL,
              "per-kernel timing records events: turn it off for the no-allocation call");
  Carver sizer(nullptr);
  ReduceWs w;
  reduce_plan(n_cap, n_seg, sizer, &w);
  KPA_REQUIRE(sizer.used <= REDUCE_SCRATCH_BYTES, KPA_EUNSUPPORTED,
              "n_cap %llu with %u segments needs %zu bytes of scratch; the static array holds "
              "%zu (about 2^29 entries over a few segments)",
              (unsigned long long)n_cap, n_seg, sizer.used, REDUCE_SCRATCH_BYTES);
  void* base = nullptr;
  KPA_CHECK(scratch_ptr(&base));
  Carver c(base);
  reduce_plan(n_cap, n_seg, c, &w);
  ReduceOut o{out_gkey, out_cnt, out_sum, out_max, out_gstart, out_gseg_off};
  return reduce_launch(keys, rids, seg_off, n_seg, static_cast<const unsigned char*>(rows),
                       layout, need_val, o, w, stream);
}

kpa_status kpa_topk_by_sum_workspace_size(uint64_t g_cap, uint32_t n_seg, size_t* bytes) {
  clear_error();
  KPA_REQUIRE(bytes, KPA_EINVAL, "bytes is null");
  Carver c(nullptr);
  TopkWs w;
  topk_plan(g_cap, n_seg ? n_seg : 1, c, &w);
  *bytes = c.used + 256;
  return KPA_OK;
}

kpa_status kpa_topk_by_sum(const uint64_t* gkey, const uint64_t* gsum, const uint64_t* gseg_off,
                           uint32_t n_seg, uint64_t g_cap, uint32_t k, uint64_t* out_key,
                           uint64_t* out_sum, uint32_t* out_n, void* ws, size_t ws_bytes,
                           hipStream_t stream) {
  clear_error();
  KPA_REQUIRE(k >= 1 && k <= TOPK_MAX, KPA_EUNSUPPORTED, "k must be in [1, 16]");
  if (n_seg == 0) return KPA_OK;
  KPA_REQUIRE(gkey && gsum && gseg_off && out_key && out_sum && out_n && ws, KPA_EINVAL,
              "null pointer");
  KPA_REQUIRE(aligned(ws, 256), KPA_EINVAL, "misaligned workspace");
  Carver c(ws);
  TopkWs w;
  topk_plan(g_cap, n_seg, c, &w);
  KPA_REQUIRE(c.used <= ws_bytes, KPA_EWORKSPACE, "workspace too small: need %zu bytes", c.used);
  KPA_CHECK(launch_seg_tiles(gseg_off, nullptr, n_seg, GT, w.tile_start, stream));
  KPA_CHECK(launch_tile_seg(w.tile_start, n_seg, nullptr, w.max_tiles, w.tile_seg, stream));
  KPA_LAUNCH("topk_local", k_topk_local, dim3((u32)w.max_tiles), dim3(BLOCK), 0, stream, gkey, gsum,
                     gseg_off, w.tile_start, w.tile_seg, n_seg, k, w.cs, w.ck, w.cn);
  KPA_LAUNCH("topk_final", k_topk_final, dim3(n_seg), dim3(BLOCK), 0, stream, w.cs, w.ck, w.cn,
                     w.tile_start, k, out_key, out_sum, out_n);
  return KPA_OK;
}

}  // extern "C"
