// Segmented stable LSD sort engine over 8-bit digits produced by a digit
// function DF (key bytes for the radix sort; bytes of a model's bucket id for
// the learned-splitter sort).
//
// DF must provide: PASSES (number of 8-bit digits), SMEM (floats of LDS it
// may use), a Params type, a device constructor DF(params, segment),
// bind(lds) called by all threads before use (then a barrier), digit(key,
// pass) -> [0, 256) and digits(key, d[PASSES]).
#pragma once

#include "sort_internal.hpp"

namespace kpa {

constexpr int HIST_TILES_PER_BLOCK = 8;

struct DigitSortBufs {
  const u64* keys_in;
  const u32* rids_in;
  u64* keys_out;
  u32* rids_out;
  u64* keys_tmp;
  u32* rids_tmp;
  u32* hist;        // n_seg * PASSES * 256
  u32* seg_mask;
  u32* tile_start;
  u32* status0;
  u32* status1;
  u32* counters;
  u64 max_tiles;
};

__device__ __forceinline__ void seg_tile_range(const SegList& sl, const u32* tile_start,
                                               u32 n_seg, u32 tile, u32& seg, u32& t_in,
                                               u64& a, u64& b, u64& base, u32& cnt) {
  seg = find_seg(tile_start, n_seg, tile);
  t_in = tile - tile_start[seg];
  a = sl.lo[seg];
  b = sl.hi[seg];
  base = a + (u64)t_in * TILE;
  cnt = base < b ? (u32)min<u64>(TILE, b - base) : 0u;
}

template <class DF>
__global__ void __launch_bounds__(BLOCK) k_ds_hist(const u64* __restrict__ keys, SegList sl,
                                                   const u32* __restrict__ tile_start,
                                                   typename DF::Params prm,
                                                   u32* __restrict__ hist) {
  __shared__ u32 h[DF::PASSES][RADIX];
  __shared__ float dfsm[DF::SMEM];
  const u32 tid = threadIdx.x;
  const u32 n_seg = sl.n();
  const u32 total = tile_start[n_seg];
  for (u32 t0 = blockIdx.x * HIST_TILES_PER_BLOCK; t0 < total;
       t0 += gridDim.x * HIST_TILES_PER_BLOCK) {
    const u32 t1 = min(total, t0 + HIST_TILES_PER_BLOCK);
    __syncthreads();
    for (int p = 0; p < DF::PASSES; ++p) h[p][tid] = 0;
    u32 cur = find_seg(tile_start, n_seg, t0);
    __syncthreads();
    for (u32 t = t0; t < t1; ++t) {
      while (cur + 1 < n_seg && tile_start[cur + 1] <= t) {
        __syncthreads();
        for (int p = 0; p < DF::PASSES; ++p) {
          const u32 c = h[p][tid];
          if (c) atomicAdd(&hist[((u64)cur * DF::PASSES + p) * RADIX + tid], c);
          h[p][tid] = 0;
        }
        __syncthreads();
        ++cur;
      }
      DF df(prm, cur);
      __syncthreads();
      df.bind(dfsm);
      __syncthreads();
      const u64 a = sl.lo[cur], b = sl.hi[cur];
      const u64 base = a + (u64)(t - tile_start[cur]) * TILE;
      const u64 end = min(b, base + TILE);
      for (u64 i = base + tid; i < end; i += BLOCK) {
        const u64 k = keys[i];
        u32 dg[DF::PASSES];
        df.digits(k, dg);
#pragma unroll
        for (int p = 0; p < DF::PASSES; ++p) atomicAdd(&h[p][dg[p]], 1u);
      }
    }
    __syncthreads();
    for (int p = 0; p < DF::PASSES; ++p) {
      const u32 c = h[p][tid];
      if (c) atomicAdd(&hist[((u64)cur * DF::PASSES + p) * RADIX + tid], c);
    }
  }
}

// Zeroes what the sort of the device-counted segments needs: their digit
// counts, the first look-back buffer for their tiles, the tile counters.
template <int UNUSED = 0>
__global__ void __launch_bounds__(BLOCK) k_ds_prepare(SegList sl, const u32* __restrict__ tile_start,
                                                      u32* __restrict__ hist, u32 hist_passes,
                                                      u32* __restrict__ status0,
                                                      u32* __restrict__ counters) {
  const u32 n_seg = sl.n();
  const u64 nh = hist ? (u64)n_seg * hist_passes * RADIX : 0ull;
  const u64 ns = (u64)tile_start[n_seg] * RADIX;
  const u64 stride = (u64)gridDim.x * BLOCK;
  for (u64 i = (u64)blockIdx.x * BLOCK + threadIdx.x; i < nh; i += stride) hist[i] = 0;
  for (u64 i = (u64)blockIdx.x * BLOCK + threadIdx.x; i < ns; i += stride) status0[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x < 16) counters[threadIdx.x] = 0;
}

// One workgroup per segment: counts -> exclusive offsets, and the mask of the
// passes whose digit varies within the segment.
template <class DF>
__global__ void __launch_bounds__(BLOCK) k_ds_scan(SegList sl, u32* __restrict__ hist,
                                                   u32* __restrict__ seg_mask) {
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
    // left untouched (mask bit 31) rather than sorted wrongly.
    if (threadIdx.x == 0) seg_mask[s] = n >= MAX_SEG_ENTRIES ? SEG_UNSUPPORTED : mask;
    __syncthreads();
  }
}

// Persistent: each workgroup claims tiles in increasing order until none is
// left.  A tile only waits (look-back) on tiles claimed earlier by running
// workgroups, so every wait ends.
template <class DF>
__global__ void __launch_bounds__(BLOCK) k_ds_pass(DigitSortBufs bf, SegList sl,
                                                   typename DF::Params prm, u32 pass,
                                                   u32* __restrict__ status_cur,
                                                   u32* __restrict__ status_next,
                                                   u32* __restrict__ counter) {
  __shared__ OnesweepSmem sm;
  __shared__ float dfsm[DF::SMEM];
  const u32 tid = threadIdx.x;
  const u32 n_seg = sl.n();
  const u32 total = bf.tile_start[n_seg];
  while (true) {
    __syncthreads();
    if (tid == 0) sm.tile = atomicAdd(counter, 1u);
    __syncthreads();
    const u32 tile = sm.tile;
    if (tile >= total) return;
    status_next[(u64)tile * RADIX + tid] = 0;  // ready for the next pass

    u32 seg, t_in, cnt;
    u64 a, b, base;
    seg_tile_range(sl, bf.tile_start, n_seg, tile, seg, t_in, a, b, base, cnt);
    const u32 mask = bf.seg_mask[seg];
    if (mask & SEG_UNSUPPORTED) continue;
    const u32 k = __popc(mask);
    if (k == 0) {
      if (pass == 0 && bf.keys_in != bf.keys_out) {
        for (u32 i = tid; i < cnt; i += BLOCK) {
          bf.keys_out[base + i] = bf.keys_in[base + i];
          bf.rids_out[base + i] = bf.rids_in[base + i];
        }
      }
      continue;
    }
    if (!((mask >> pass) & 1)) continue;
    const u32 q = __popc(mask & ((1u << pass) - 1));
    const u64* src_k = q == 0 ? bf.keys_in : (((k - q) & 1) == 0 ? bf.keys_out : bf.keys_tmp);
    const u32* src_r = q == 0 ? bf.rids_in : (((k - q) & 1) == 0 ? bf.rids_out : bf.rids_tmp);
    u64* dst_k = ((k - 1 - q) & 1) == 0 ? bf.keys_out : bf.keys_tmp;
    u32* dst_r = ((k - 1 - q) & 1) == 0 ? bf.rids_out : bf.rids_tmp;

    DF df(prm, seg);
    df.bind(dfsm);
    __syncthreads();
    u64 kk[ITEMS];
    u32 rr[ITEMS], dd[ITEMS];
    u32 valid = 0;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const u32 o = tile_offset(j);
      if (o < cnt) {
        kk[j] = src_k[base + o];
        rr[j] = src_r[base + o];
        valid |= 1u << j;
      } else {
        kk[j] = 0;
        rr[j] = 0;
      }
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) dd[j] = ((valid >> j) & 1) ? df.digit(kk[j], pass) : 0u;
    const u64 my_base = a + bf.hist[((u64)seg * DF::PASSES + pass) * RADIX + tid];
    onesweep_tile(sm, kk, rr, dd, valid, status_cur, tile, t_in, my_base, dst_k, dst_r);
  }
}

// Workgroups that fit on the device at once for a kernel (persistent grids).
template <class K>
u32 resident_grid(K kernel, u32 cap) {
  static u32 cached = 0;
  if (!cached) {
    int dev = 0, per_cu = 1;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return cap;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, BLOCK, 0) != hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    cached = (u32)(p.multiProcessorCount * per_cu);
  }
  return cached < cap ? cached : cap;
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
             with_hist ? b.hist : nullptr, (u32)DF::PASSES, b.status0, b.counters);
  if (with_hist) {
    const u32 hist_blocks = (u32)std::min<u64>(ceil_div(b.max_tiles, HIST_TILES_PER_BLOCK), 4096);
    KPA_LAUNCH(radix ? "radix_hist" : "learned_hist", k_ds_hist<DF>, dim3(hist_blocks),
               dim3(BLOCK), 0, st, b.keys_in, sl, b.tile_start, prm, b.hist);
    KPA_LAUNCH(radix ? "radix_scan" : "learned_scan", k_ds_scan<DF>,
               dim3(std::min<u32>(sl.n_max, 2048)), dim3(BLOCK), 0, st, sl, b.hist, b.seg_mask);
  }
#ifdef KPA_ONE_TILE_PER_BLOCK
  const u32 grid = (u32)b.max_tiles;
#else
  const u32 grid = resident_grid(k_ds_pass<DF>, (u32)std::min<u64>(b.max_tiles, 1u << 20));
#endif
  const char* pname = radix ? "radix_pass" : (DF::PASSES == 2 ? "learned_scatter" : "pivot_scatter");
  for (u32 p = 0; p < (u32)DF::PASSES; ++p) {
    u32* cur = (p & 1) ? b.status1 : b.status0;
    u32* nxt = (p & 1) ? b.status0 : b.status1;
    KPA_LAUNCH(pname, k_ds_pass<DF>, dim3(grid), dim3(BLOCK), 0, st, b, sl, prm, p, cur, nxt,
               b.counters + p);
  }
  return KPA_OK;
}

}  // namespace kpa
