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
#include "onesweep.hpp"
#include "sort_internal.hpp"

namespace kpa {

constexpr int HIST_TILES_PER_BLOCK = 8;

// 8 digit histograms per segment, accumulated in LDS and flushed with global
// atomics whenever the block moves to the next segment.
__global__ void __launch_bounds__(BLOCK) k_radix_hist(const u64* __restrict__ keys,
                                                      const u64* __restrict__ seg_off,
                                                      const u32* __restrict__ tile_start,
                                                      u32 n_seg, u32* __restrict__ hist) {
  __shared__ u32 h[8][RADIX];
  const u32 tid = threadIdx.x;
  const u32 total = tile_start[n_seg];
  u32 t0 = blockIdx.x * HIST_TILES_PER_BLOCK;
  if (t0 >= total) return;
  u32 t1 = min(total, t0 + HIST_TILES_PER_BLOCK);
  for (int p = 0; p < 8; ++p) h[p][tid] = 0;
  u32 cur = find_seg(tile_start, n_seg, t0);
  __syncthreads();
  for (u32 t = t0; t < t1; ++t) {
    while (cur + 1 < n_seg && tile_start[cur + 1] <= t) {
      // flush the finished segment
      __syncthreads();
      for (int p = 0; p < 8; ++p) {
        u32 c = h[p][tid];
        if (c) atomicAdd(&hist[((u64)cur * 8 + p) * RADIX + tid], c);
        h[p][tid] = 0;
      }
      __syncthreads();
      ++cur;
    }
    const u64 a = seg_off[cur], b = seg_off[cur + 1];
    const u64 base = a + (u64)(t - tile_start[cur]) * TILE;
    const u64 end = min(b, base + TILE);
    for (u64 i = base + tid; i < end; i += BLOCK) {
      u64 k = keys[i];
#pragma unroll
      for (int p = 0; p < 8; ++p) atomicAdd(&h[p][(k >> (8 * p)) & 255], 1u);
    }
  }
  __syncthreads();
  for (int p = 0; p < 8; ++p) {
    u32 c = h[p][tid];
    if (c) atomicAdd(&hist[((u64)cur * 8 + p) * RADIX + tid], c);
  }
}

// One workgroup per segment: counts -> exclusive offsets, and the mask of
// passes whose digit varies.
__global__ void __launch_bounds__(BLOCK) k_radix_scan(const u64* __restrict__ seg_off,
                                                      u32* __restrict__ hist,
                                                      u32* __restrict__ seg_mask,
                                                      u32 pass_lo, u32 pass_hi) {
  __shared__ u32 sc[WAVES + 1];
  const u32 s = blockIdx.x;
  const u64 n = seg_off[s + 1] - seg_off[s];
  u32 mask = 0;
  for (u32 p = pass_lo; p < pass_hi; ++p) {
    u32* hp = hist + ((u64)s * 8 + p) * RADIX;
    const u32 c = hp[threadIdx.x];
    u32 tot;
    const u32 ex = block_excl_sum(c, sc, &tot);
    hp[threadIdx.x] = ex;
    const int constant = __syncthreads_or(c == n);
    if (!constant) mask |= 1u << p;
  }
  // Segments of 2^30 or more entries exceed the look-back word; they are left
  // untouched (mask bit 31) rather than sorted wrongly.
  if (threadIdx.x == 0) seg_mask[s] = n >= MAX_SEG_ENTRIES ? SEG_UNSUPPORTED : mask;
}

__global__ void __launch_bounds__(BLOCK) k_radix_pass(
    const u64* __restrict__ keys_in, const u32* __restrict__ rids_in, u64* __restrict__ keys_out,
    u32* __restrict__ rids_out, u64* __restrict__ keys_tmp, u32* __restrict__ rids_tmp,
    const u64* __restrict__ seg_off, const u32* __restrict__ tile_start, u32 n_seg,
    const u32* __restrict__ seg_mask, const u32* __restrict__ digit_off, u32 pass,
    u32* __restrict__ status_cur, u32* __restrict__ status_next, u32* __restrict__ counter) {
  __shared__ OnesweepSmem sm;
  const u32 tid = threadIdx.x;
  if (tid == 0) sm.tile = atomicAdd(counter, 1u);
  __syncthreads();
  const u32 tile = sm.tile;
  if (tile >= tile_start[n_seg]) return;
  status_next[(u64)tile * RADIX + tid] = 0;  // ready for the next pass

  const u32 seg = find_seg(tile_start, n_seg, tile);
  const u32 t_in = tile - tile_start[seg];
  const u64 a = seg_off[seg], b = seg_off[seg + 1];
  const u64 base = a + (u64)t_in * TILE;
  const u32 cnt = base < b ? (u32)min<u64>(TILE, b - base) : 0u;
  const u32 mask = seg_mask[seg];
  if (mask & SEG_UNSUPPORTED) return;
  const u32 k = __popc(mask);
  if (k == 0) {
    if (pass == 0) {
      for (u32 i = tid; i < cnt; i += BLOCK) {
        keys_out[base + i] = keys_in[base + i];
        rids_out[base + i] = rids_in[base + i];
      }
    }
    return;
  }
  if (!((mask >> pass) & 1)) return;
  const u32 q = __popc(mask & ((1u << pass) - 1));
  const u64* src_k = q == 0 ? keys_in : (((k - q) & 1) == 0 ? keys_out : keys_tmp);
  const u32* src_r = q == 0 ? rids_in : (((k - q) & 1) == 0 ? rids_out : rids_tmp);
  u64* dst_k = ((k - 1 - q) & 1) == 0 ? keys_out : keys_tmp;
  u32* dst_r = ((k - 1 - q) & 1) == 0 ? rids_out : rids_tmp;

  u64 kk[ITEMS];
  u32 rr[ITEMS], dd[ITEMS];
  u32 valid = 0;
  const u32 shift = 8 * pass;
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
    dd[j] = (u32)(kk[j] >> shift) & 255u;
  }
  const u64 my_base = a + digit_off[((u64)seg * 8 + pass) * RADIX + tid];
  onesweep_tile(sm, kk, rr, dd, valid, status_cur, tile, t_in == 0, my_base, dst_k, dst_r);
}

kpa_status radix_sort_plan(u64 n_cap, u32 n_seg, Carver& c, RadixWs* w) {
  const u64 tiles = max_tiles(n_cap, n_seg, TILE);
  w->keys_tmp = c.take<u64>(n_cap);
  w->rids_tmp = c.take<u32>(n_cap);
  w->hist = c.take<u32>((u64)n_seg * 8 * RADIX);
  w->seg_mask = c.take<u32>(n_seg);
  w->tile_start = c.take<u32>((u64)n_seg + 1);
  w->status0 = c.take<u32>(tiles * RADIX);
  w->status1 = c.take<u32>(tiles * RADIX);
  w->counters = c.take<u32>(16);
  w->max_tiles = tiles;
  return KPA_OK;
}

kpa_status radix_sort_launch(const u64* keys_in, const u32* rids_in, u64* keys_out,
                             u32* rids_out, const u64* seg_off, u32 n_seg, const RadixWs& w,
                             hipStream_t st) {
  KPA_CHECK(launch_seg_tiles(seg_off, nullptr, n_seg, TILE, w.tile_start, st));
  KPA_CHECK(launch_fill_u32(w.hist, (u64)n_seg * 8 * RADIX, 0, st));
  KPA_CHECK(launch_fill_u32(w.counters, 16, 0, st));
  KPA_CHECK(launch_fill_u32(w.status0, w.max_tiles * RADIX, 0, st));
  const u32 hist_blocks = (u32)ceil_div(w.max_tiles, HIST_TILES_PER_BLOCK);
  hipLaunchKernelGGL(k_radix_hist, dim3(hist_blocks), dim3(BLOCK), 0, st, keys_in, seg_off,
                     w.tile_start, n_seg, w.hist);
  KPA_LAUNCHED();
  hipLaunchKernelGGL(k_radix_scan, dim3(n_seg), dim3(BLOCK), 0, st, seg_off, w.hist, w.seg_mask,
                     0u, 8u);
  KPA_LAUNCHED();
  for (u32 p = 0; p < 8; ++p) {
    u32* cur = (p & 1) ? w.status1 : w.status0;
    u32* nxt = (p & 1) ? w.status0 : w.status1;
    hipLaunchKernelGGL(k_radix_pass, dim3((u32)w.max_tiles), dim3(BLOCK), 0, st, keys_in,
                       rids_in, keys_out, rids_out, w.keys_tmp, w.rids_tmp, seg_off, w.tile_start,
                       n_seg, w.seg_mask, w.hist, p, cur, nxt, w.counters + p);
    KPA_LAUNCHED();
  }
  return KPA_OK;
}

}  // namespace kpa
