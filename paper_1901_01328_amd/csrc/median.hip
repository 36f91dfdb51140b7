// Median per key (Sec. 6 "Windowed Median Per Key"; a percentile by key is a
// sort followed by a reduction, Sec. 4.2).  For each run of equal keys in a
// sorted KPA, the lower median v[(c-1)/2] of its c values in ascending order.
//
// Runs come from the keyed reduction (key, count, first entry).  Selection
// by size class:
//   c <= 16   one thread: values in registers, counting selection;
//   c <= 4096 one workgroup: values in LDS, bitonic sort;
//   larger    one workgroup: radix selection over the value's 8 bytes, most
//             significant first (a histogram of the candidates per byte).
#include "reduce_internal.hpp"

namespace kpa {

constexpr u32 MED_SMALL = 16;
constexpr u32 MED_BINS = 256;
constexpr u32 MED_MID = 4096;

struct MedSrc {
  const u32* rids;
  const unsigned char* rows;
  u32 row_bytes, val_off, val_w;
  __device__ __forceinline__ u64 val(u64 entry) const {
    return load_val(rows, rids[entry], row_bytes, val_off, val_w);
  }
};

__global__ void __launch_bounds__(BLOCK) k_median_small(MedSrc src, const u64* __restrict__ gcnt,
                                                        const u64* __restrict__ gstart,
                                                        const u64* __restrict__ gseg_off, u32 n_seg,
                                                        u64* __restrict__ out_med,
                                                        u32* __restrict__ mid_list,
                                                        u32* __restrict__ mid_count,
                                                        u32* __restrict__ big_list,
                                                        u32* __restrict__ big_count,
                                                        u64* __restrict__ out_sum) {
  const u64 G = gseg_off[n_seg];
  for (u64 g = (u64)blockIdx.x * BLOCK + threadIdx.x; g < G; g += (u64)gridDim.x * BLOCK) {
    const u64 c = gcnt[g], s = gstart[g];
    if (c > MED_SMALL) {
      if (c <= MED_MID) mid_list[atomicAdd(mid_count, 1u)] = (u32)g;
      else big_list[atomicAdd(big_count, 1u)] = (u32)g;
      continue;
    }
    u64 v[MED_SMALL];
#pragma unroll
    for (u32 i = 0; i < MED_SMALL; ++i) v[i] = i < c ? src.val(s + i) : ~0ull;
    if (out_sum) {
      u64 sum = 0;
#pragma unroll
      for (u32 i = 0; i < MED_SMALL; ++i) sum += i < c ? v[i] : 0ull;
      out_sum[g] = sum;
    }
    const u32 h = (u32)(c - 1) / 2;
    u64 med = 0;
#pragma unroll
    for (u32 a = 0; a < MED_SMALL; ++a) {
      u32 less = 0, le = 0;
#pragma unroll
      for (u32 b = 0; b < MED_SMALL; ++b) {
        less += (b < c) & (v[b] < v[a]);
        le += (b < c) & (v[b] <= v[a]);
      }
      if (a < c && less <= h && h < le) med = v[a];
    }
    out_med[g] = med;
  }
}

__global__ void __launch_bounds__(BLOCK) k_median_mid(MedSrc src, const u64* __restrict__ gcnt,
                                                      const u64* __restrict__ gstart,
                                                      const u32* __restrict__ list,
                                                      const u32* __restrict__ count,
                                                      u64* __restrict__ out_med,
                                                      u64* __restrict__ out_sum) {
  __shared__ u64 v[MED_MID];
  __shared__ u64 red[WAVES];
  const u32 n = *count;
  for (u32 q = blockIdx.x; q < n; q += gridDim.x) {
    const u32 g = list[q];
    const u32 c = (u32)gcnt[g];
    const u64 s = gstart[g];
    u32 p2 = 1;
    while (p2 < c) p2 <<= 1;
    __syncthreads();
    u64 part = 0;  // this thread's share of the group's sum
    for (u32 i = threadIdx.x; i < p2; i += BLOCK) {
      const u64 x = i < c ? src.val(s + i) : ~0ull;
      v[i] = x;
      part += i < c ? x : 0ull;
    }
    if (out_sum) {  // uniform
      part = wave_sum(part);
      if (__lane_id() == 0) red[threadIdx.x >> 6] = part;
    }
    __syncthreads();
    if (out_sum && threadIdx.x == 0) {
      u64 sum = 0;
      for (int w = 0; w < WAVES; ++w) sum += red[w];
      out_sum[g] = sum;
    }
    // bitonic sort of p2 values, ascending
    for (u32 k = 2; k <= p2; k <<= 1) {
      for (u32 j = k >> 1; j > 0; j >>= 1) {
        for (u32 i = threadIdx.x; i < p2; i += BLOCK) {
          const u32 x = i ^ j;
          if (x > i) {
            const u64 a = v[i], b = v[x];
            const bool up = (i & k) == 0;
            if ((a > b) == up) {
              v[i] = b;
              v[x] = a;
            }
          }
        }
        __syncthreads();
      }
    }
    if (threadIdx.x == 0) out_med[g] = v[(c - 1) / 2];
  }
}

__global__ void __launch_bounds__(BLOCK) k_median_big(MedSrc src, const u64* __restrict__ gcnt,
                                                      const u64* __restrict__ gstart,
                                                      const u32* __restrict__ list,
                                                      const u32* __restrict__ count,
                                                      u64* __restrict__ out_med,
                                                      u64* __restrict__ out_sum) {
  __shared__ u32 h[MED_BINS];
  __shared__ u64 sel[2];
  __shared__ u64 red[WAVES];
  const u32 n = *count;
  for (u32 q = blockIdx.x; q < n; q += gridDim.x) {
    const u32 g = list[q];
    const u64 c = gcnt[g], s = gstart[g];
    u64 prefix = 0, rank = (c - 1) / 2;
    u64 part = 0;  // this thread's share of the group's sum (first byte pass)
    for (int byte = 7; byte >= 0; --byte) {
      const u32 shift = 8 * byte;
      const u64 himask = byte == 7 ? 0ull : (~0ull << (shift + 8));
      __syncthreads();
      h[threadIdx.x] = 0;
      __syncthreads();
      for (u64 i = threadIdx.x; i < c; i += BLOCK) {
        const u64 x = src.val(s + i);
        if (byte == 7) part += x;
        if ((x & himask) == prefix) atomicAdd(&h[(x >> shift) & 255], 1u);
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        u64 acc = 0;
        u32 d = 0;
        for (; d < MED_BINS; ++d) {
          if (rank < acc + h[d]) break;
          acc += h[d];
        }
        sel[0] = prefix | ((u64)d << shift);
        sel[1] = rank - acc;
      }
      __syncthreads();
      prefix = sel[0];
      rank = sel[1];
    }
    if (threadIdx.x == 0) out_med[g] = prefix;
    if (out_sum) {  // uniform; red is read by thread 0 only after the barrier
      part = wave_sum(part);
      if (__lane_id() == 0) red[threadIdx.x >> 6] = part;
      __syncthreads();
      if (threadIdx.x == 0) {
        u64 sum = 0;
        for (int w = 0; w < WAVES; ++w) sum += red[w];
        out_sum[g] = sum;
      }
    }
  }
}

struct MedianWs {
  ReduceWs red;
  u64* gcnt;
  u64* gstart;
  u32* mid_list;
  u32* big_list;
  u32* counts;
};

static void median_plan(u64 n_cap, u32 n_seg, Carver& c, MedianWs* w) {
  reduce_plan(n_cap, n_seg, c, &w->red);
  const u64 cap = n_cap ? n_cap : 1;
  w->gcnt = c.take<u64>(cap);
  w->gstart = c.take<u64>(cap);
  w->mid_list = c.take<u32>(cap / (MED_SMALL + 1) + 1);
  w->big_list = c.take<u32>(cap / (MED_MID + 1) + 1);
  w->counts = c.take<u32>(2);
}

}  // namespace kpa

using namespace kpa;

extern "C" {

kpa_status kpa_median_by_key_workspace_size(uint64_t n_cap, uint32_t n_seg, size_t* bytes) {
  clear_error();
  KPA_REQUIRE(bytes, KPA_EINVAL, "bytes is null");
  Carver c(nullptr);
  MedianWs w;
  median_plan(n_cap, n_seg ? n_seg : 1, c, &w);
  *bytes = c.used + 256;
  return KPA_OK;
}

kpa_status kpa_median_by_key(const uint64_t* keys, const uint32_t* rids, const uint64_t* seg_off,
                             uint32_t n_seg, uint64_t n_cap, const void* rows,
                             const kpa_row_layout* layout, uint64_t* out_gkey, uint64_t* out_med,
                             uint64_t* out_gseg_off, uint64_t* out_cnt, uint64_t* out_sum,
                             void* ws, size_t ws_bytes, hipStream_t stream) {
  clear_error();
  KPA_CHECK(check_layout(layout, true, false));
  if (n_seg == 0) return KPA_OK;
  KPA_REQUIRE(keys && rids && seg_off && rows && out_gkey && out_med && out_gseg_off && ws,
              KPA_EINVAL, "null pointer");
  KPA_REQUIRE(aligned(keys, 8) && aligned(rids, 4) && aligned(rows, 16) && aligned(out_med, 8) &&
                  aligned(out_gkey, 8) && aligned(out_gseg_off, 8) && aligned(ws, 256) &&
                  aligned(out_cnt, 8) && aligned(out_sum, 8),
              KPA_EINVAL, "misaligned pointer");
  KPA_REQUIRE(n_cap < (1ull << 32), KPA_EUNSUPPORTED, "n_cap must be below 2^32");
  Carver c(ws);
  MedianWs w;
  median_plan(n_cap, n_seg, c, &w);
  KPA_REQUIRE(c.used <= ws_bytes, KPA_EWORKSPACE, "workspace too small: need %zu bytes", c.used);
  u64* gcnt = out_cnt ? out_cnt : w.gcnt;  // the counts go where the caller wants them
  ReduceOut o{out_gkey, gcnt, nullptr, nullptr, w.gstart, out_gseg_off};
  KPA_CHECK(reduce_launch(keys, rids, seg_off, n_seg, nullptr, nullptr, false, o, w.red, stream));
  KPA_CHECK(launch_fill_u32(w.counts, 2, 0, stream));
  MedSrc src{rids, static_cast<const unsigned char*>(rows), layout->row_bytes, layout->val_off,
             layout->val_w};
  const u32 grid = (u32)std::min<u64>(ceil_div(n_cap ? n_cap : 1, BLOCK), 8192);
  KPA_LAUNCH("median_small", k_median_small, dim3(grid), dim3(BLOCK), 0, stream, src, gcnt,
             w.gstart, out_gseg_off, n_seg, out_med, w.mid_list, w.counts, w.big_list,
             w.counts + 1, out_sum);
  KPA_LAUNCH("median_mid", k_median_mid, dim3(2048), dim3(BLOCK), 0, stream, src, gcnt, w.gstart,
             w.mid_list, w.counts, out_med, out_sum);
  KPA_LAUNCH("median_big", k_median_big, dim3(512), dim3(BLOCK), 0, stream, src, gcnt, w.gstart,
             w.big_list, w.counts + 1, out_med, out_sum);
  return KPA_OK;
}

}  // extern "C"
