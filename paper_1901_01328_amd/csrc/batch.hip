// Batched sort of many segments of uneven size (the windows of many
// substreams) in a fixed sequence of launches whose sizes are all read from
// device memory, so that one captured graph serves every batch of the same
// segment count and capacity.  The paper's runtime gets its parallelism from
// many bundles and windows in flight at once (Sec. 3, data parallelism over
// bundles, out-of-order bundle processing); here one batch holds all of them.
//
// Segments are split by size into three classes:
//   small  n <= small_cap (<= 4096): one workgroup loads the segment into LDS,
//          sorts it there (stable LSD over the bytes that vary) and writes it;
//   mid    small_cap < n <= mid_cap: one workgroup runs the LSD radix passes
//          itself through device memory: one read for the varying bytes, one
//          for their digit counts, then per varying byte a stable scatter of
//          the segment's tiles in order (no cross-workgroup look-back);
//   large  n > mid_cap: the multi-workgroup onesweep radix sort, or the
//          learned-splitter sort, over the large segments only.
// A single-workgroup classifier writes the work table (small and mid segment
// ids, largest first) and the large-segment list; one persistent kernel
// drains the table.  Every class produces the stable sort, so the output is
// the same whatever the class boundaries.
#include "learned_internal.hpp"
#include "onchip_sort.hpp"
#include "sort_internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

namespace kpa {
namespace {

struct BatchSmem {
  static constexpr int kWaves = WAVES;
  u32 whist[WAVES][RADIX];
  u32 lstart[RADIX];
  u64 gbase[RADIX];
  u32 scan[WAVES + 1];
  u32 red[WAVES];
  u64 red64[2 * WAVES];
  u32 dh[8][RADIX];  // mid class: digit counts, then running destinations
  u32 item;
  u32 count;
  u64 skeys[TILE];
  u32 srids[TILE];
  unsigned char sdig[TILE];
};

struct BatchWs {
  u64* large_lo;  // n_seg: [lo, hi) of large segments, empty for the rest
  u64* large_hi;
  u32* items;     // n_seg: small and mid segment ids, largest first
  u32* n_items;   // 1
  u32* counter;   // 1: next work-table item
  u64* keys_tmp;  // ping-pong buffer of the mid class (from the large path's plan)
  u32* rids_tmp;
  u64* vals_tmp;  // the same for a value column (null without one)
  RadixWs rw;
  LearnedWs lw;
};

constexpr int SIZE_BINS = 33;

// One workgroup: classify, and order the table by floor(log2(n)) descending
// so that the longest items start first.
__global__ void __launch_bounds__(1024) k_batch_classify(const u64* __restrict__ off, u32 n_seg,
                                                         u32 mid_cap,
                                                         u64* __restrict__ large_lo,
                                                         u64* __restrict__ large_hi,
                                                         u32* __restrict__ items,
                                                         u32* __restrict__ n_items,
                                                         u32* __restrict__ counter) {
  __shared__ u32 bins[SIZE_BINS];
  const u32 tid = threadIdx.x;
  if (tid < SIZE_BINS) bins[tid] = 0;
  __syncthreads();
  for (u32 s = tid; s < n_seg; s += blockDim.x) {
    const u64 a = off[s], b = off[s + 1];
    const u64 n = b - a;
    const bool large = n > mid_cap;
    large_lo[s] = a;
    large_hi[s] = large ? b : a;
    if (!large && n > 0) atomicAdd(&bins[63 - __clzll(n)], 1u);
  }
  __syncthreads();
  if (tid == 0) {
    u32 acc = 0;
    for (int i = SIZE_BINS - 1; i >= 0; --i) {
      const u32 c = bins[i];
      bins[i] = acc;
      acc += c;
    }
    *n_items = acc;
    *counter = 0;
  }
  __syncthreads();
  for (u32 s = tid; s < n_seg; s += blockDim.x) {
    const u64 n = off[s + 1] - off[s];
    if (n > 0 && n <= mid_cap) items[atomicAdd(&bins[63 - __clzll(n)], 1u)] = s;
  }
}

// Small class: the whole segment in LDS.  With a value column the on-chip
// sort orders local indices, and row ids and values are gathered through
// them from the segment's input (a few KB, in cache).
template <bool VALS>
__device__ void small_sort(BatchSmem& sm, const u64* __restrict__ keys_in,
                           const u32* __restrict__ rids_in, const u64* __restrict__ vals_in,
                           u64* __restrict__ keys_out, u32* __restrict__ rids_out,
                           u64* __restrict__ vals_out, u64 a, u32 n) {
  const u32 tid = threadIdx.x;
  for (u32 i = tid; i < n; i += BLOCK) {
    sm.skeys[i] = keys_in[a + i];
    sm.srids[i] = VALS ? i : (rids_in ? rids_in[a + i] : (u32)(a + i));
  }
  lds_sort(sm, n);  // begins with a barrier; leaves the result (or the input) in sm
  __syncthreads();
  for (u32 i = tid; i < n; i += BLOCK) {
    keys_out[a + i] = sm.skeys[i];
    if (VALS) {
      const u32 o = sm.srids[i];
      rids_out[a + i] = rids_in ? rids_in[a + o] : (u32)(a + o);
      vals_out[a + i] = vals_in[a + o];
    } else {
      rids_out[a + i] = sm.srids[i];
    }
  }
}

// Mid class: LSD radix over the varying bytes by one workgroup.  With a
// value column each tile's values follow its keys through the key slots of
// LDS once the keys and row ids are written.
template <bool VALS>
__device__ void mid_sort(BatchSmem& sm, const u64* __restrict__ keys_in,
                         const u32* __restrict__ rids_in, const u64* __restrict__ vals_in,
                         u64* __restrict__ keys_out, u32* __restrict__ rids_out,
                         u64* __restrict__ vals_out, u64* __restrict__ keys_tmp,
                         u32* __restrict__ rids_tmp, u64* __restrict__ vals_tmp, u64 a, u32 n) {
  const u32 tid = threadIdx.x;
  u64 vor = 0, vand = ~0ull;
  for (u32 i = tid; i < n; i += BLOCK) {
    const u64 k = keys_in[a + i];
    vor |= k;
    vand &= k;
  }
  block_or_and(vor, vand, sm.red64);
  const u64 vary = vor ^ vand;
  u32 amask = 0;
#pragma unroll
  for (int p = 0; p < 8; ++p)
    if ((vary >> (8 * p)) & 255u) amask |= 1u << p;
  const u32 k_act = __popc(amask);
  if (k_act == 0) {  // one key: the input order is the sorted order
    for (u32 i = tid; i < n; i += BLOCK) {
      keys_out[a + i] = keys_in[a + i];
      rids_out[a + i] = rids_in ? rids_in[a + i] : (u32)(a + i);
      if (VALS) vals_out[a + i] = vals_in[a + i];
    }
    return;
  }
  for (u32 i = tid; i < 8 * RADIX; i += BLOCK) (&sm.dh[0][0])[i] = 0;
  __syncthreads();
  for (u32 i = tid; i < n; i += BLOCK) {
    const u64 k = keys_in[a + i];
#pragma unroll
    for (int p = 0; p < 8; ++p)
      if ((amask >> p) & 1) atomicAdd(&sm.dh[p][(u32)(k >> (8 * p)) & 255u], 1u);
  }
  __syncthreads();
  for (int p = 0; p < 8; ++p) {
    if (!((amask >> p) & 1)) continue;
    u32 tot;
    const u32 c = sm.dh[p][tid];
    const u32 e = block_excl_sum(c, sm.scan, &tot);
    sm.dh[p][tid] = e;
  }
  __syncthreads();

  const u32 n_tiles = (n + TILE - 1) / TILE;
  u32 q = 0;
  for (u32 p = 0; p < 8; ++p) {
    if (!((amask >> p) & 1)) continue;
    const bool first = q == 0, to_out = ((k_act - 1 - q) & 1) == 0;
    const bool from_out = ((k_act - q) & 1) == 0;
    const u64* src_k = first ? keys_in : (from_out ? keys_out : keys_tmp);
    const u32* src_r = first ? rids_in : (from_out ? rids_out : rids_tmp);
    const u64* src_v = first ? vals_in : (from_out ? vals_out : vals_tmp);
    u64* dst_k = to_out ? keys_out : keys_tmp;
    u32* dst_r = to_out ? rids_out : rids_tmp;
    u64* dst_v = to_out ? vals_out : vals_tmp;
    for (u32 t = 0; t < n_tiles; ++t) {
      const u32 cnt = min((u32)TILE, n - t * TILE);
      const u64 base = a + (u64)t * TILE;
      u64 kk[ITEMS];
      u32 rr[ITEMS], dd[ITEMS], rank[ITEMS];
      u32 valid = 0;
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) {
        const u32 o = tile_offset(j);
        if (o < cnt) {
          kk[j] = src_k[base + o];
          rr[j] = src_r ? src_r[base + o] : (u32)(base + o);  // no input rids: positions
          valid |= 1u << j;
        } else {
          kk[j] = 0;
          rr[j] = 0;
        }
        dd[j] = (u32)(kk[j] >> (8 * p)) & 255u;
      }
      __syncthreads();  // the previous tile's scatter has read sm
      u32 tile_count;
      const u32 total = rank_tile(sm.whist, sm.lstart, sm.scan, dd, valid, rank, &tile_count);
      const u32 run = sm.dh[p][tid];
      sm.gbase[tid] = a + run;
      sm.dh[p][tid] = run + total;
      if (tid == 0) sm.count = tile_count;
      __syncthreads();
      if (VALS) {
        u32 pos[ITEMS];
        stage_tile_pos<BatchSmem, ITEMS>(sm, kk, rr, dd, rank, valid, pos);
        write_staged<BatchSmem, WAVES>(sm, dst_k, dst_r);
        u64 vv[ITEMS];
#pragma unroll
        for (int j = 0; j < ITEMS; ++j)
          vv[j] = ((valid >> j) & 1) ? src_v[base + tile_offset(j)] : 0ull;
        write_staged_vals<BatchSmem, WAVES, ITEMS>(sm, vv, pos, valid, dst_v);
      } else {
        stage_scatter(sm, kk, rr, dd, rank, valid, dst_k, dst_r);
      }
    }
    ++q;
    // the next pass reads what this one wrote (other threads' stores)
    __threadfence_block();
    __syncthreads();
  }
}

template <bool VALS>
__global__ void __launch_bounds__(BLOCK, 2) k_batch_small_mid(
    const u64* __restrict__ keys_in, const u32* __restrict__ rids_in,
    const u64* __restrict__ vals_in, u64* __restrict__ keys_out, u32* __restrict__ rids_out,
    u64* __restrict__ vals_out, u64* __restrict__ keys_tmp, u32* __restrict__ rids_tmp,
    u64* __restrict__ vals_tmp, const u64* __restrict__ off, const u32* __restrict__ items,
    const u32* __restrict__ n_items, u32* __restrict__ counter, u32 small_cap) {
  __shared__ BatchSmem sm;
  const u32 total = *n_items;
  while (true) {
    __syncthreads();
    if (threadIdx.x == 0) sm.item = atomicAdd(counter, 1u);
    __syncthreads();
    const u32 it = sm.item;
    if (it >= total) return;
    const u32 s = items[it];
    const u64 a = off[s];
    const u32 n = (u32)(off[s + 1] - a);
    if (n <= small_cap)
      small_sort<VALS>(sm, keys_in, rids_in, vals_in, keys_out, rids_out, vals_out, a, n);
    else
      mid_sort<VALS>(sm, keys_in, rids_in, vals_in, keys_out, rids_out, vals_out, keys_tmp,
                     rids_tmp, vals_tmp, a, n);
  }
}

kpa_status check_config(const kpa_batch_config* cfg) {
  KPA_REQUIRE(cfg != nullptr, KPA_EINVAL, "config is null");
  KPA_REQUIRE(cfg->small_cap <= TILE, KPA_EUNSUPPORTED, "small_cap must be at most %d", TILE);
  KPA_REQUIRE(cfg->mid_cap >= cfg->small_cap && cfg->mid_cap < MAX_SEG_ENTRIES, KPA_EINVAL,
              "mid_cap must lie in [small_cap, 2^30)");
  KPA_REQUIRE(cfg->large_algo == KPA_SORT_RADIX || cfg->large_algo == KPA_SORT_LEARNED,
              KPA_EINVAL, "bad large_algo");
  KPA_REQUIRE(cfg->bucket_log2 == 0 || (cfg->bucket_log2 >= 6 && cfg->bucket_log2 <= 12),
              KPA_EINVAL, "bucket_log2 must be 0 or lie in [6, 12]");
  return KPA_OK;
}

kpa_status batch_plan(u64 n_cap, u32 n_seg, const kpa_batch_config* cfg, Carver& c, BatchWs* w,
                      bool vals = false) {
  w->large_lo = c.take<u64>(n_seg);
  w->large_hi = c.take<u64>(n_seg);
  w->items = c.take<u32>(n_seg);
  w->n_items = c.take<u32>(1);
  w->counter = c.take<u32>(1);
  if (cfg->large_algo == KPA_SORT_LEARNED) {
    KPA_CHECK(learned_sort_plan(n_cap, n_seg, c, &w->lw, vals));
    w->keys_tmp = w->lw.keys_tmp;
    w->rids_tmp = w->lw.rids_tmp;
    w->vals_tmp = w->lw.vals_tmp;
  } else {
    KPA_CHECK(radix_sort_plan(n_cap, n_seg, c, &w->rw, vals));
    w->keys_tmp = w->rw.keys_tmp;
    w->rids_tmp = w->rw.rids_tmp;
    w->vals_tmp = w->rw.vals_tmp;
  }
  return KPA_OK;
}

u32 small_mid_grid(const kpa_batch_config* cfg) {
  static u32 resident = 0;
  if (!resident) {
    int dev = 0, per_cu = 1;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess)
      return 1024;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_small_mid<false>, BLOCK, 0) !=
            hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    resident = (u32)(p.multiProcessorCount * per_cu);
  }
  return cfg->grid ? std::min<u32>(cfg->grid, 1u << 16) : resident;
}

// vals_in/vals_out: null, or a value column (the plan had vals).
kpa_status batch_launch(const u64* keys_in, const u32* rids_in, u64* keys_out, u32* rids_out,
                        const u64* seg_off, u32 n_seg, const kpa_batch_config* cfg,
                        const kpa_pwl_model* models, kpa_sort_stats* stats, const BatchWs& w,
                        hipStream_t st, const u64* vals_in = nullptr, u64* vals_out = nullptr) {
  KPA_REQUIRE(!vals_in || (vals_out && w.vals_tmp), KPA_EINVAL,
              "a value column needs an output and a planned buffer");
  KPA_LAUNCH("batch_classify", k_batch_classify, dim3(1), dim3(1024), 0, st, seg_off, n_seg,
             cfg->mid_cap, w.large_lo, w.large_hi, w.items, w.n_items,
             w.counter);
  if (vals_in)
    KPA_LAUNCH("batch_small_mid", k_batch_small_mid<true>, dim3(small_mid_grid(cfg)), dim3(BLOCK),
               0, st, keys_in, rids_in, vals_in, keys_out, rids_out, vals_out, w.keys_tmp,
               w.rids_tmp, w.vals_tmp, seg_off, w.items, w.n_items, w.counter, cfg->small_cap);
  else
    KPA_LAUNCH("batch_small_mid", k_batch_small_mid<false>, dim3(small_mid_grid(cfg)),
               dim3(BLOCK), 0, st, keys_in, rids_in, nullptr, keys_out, rids_out, nullptr,
               w.keys_tmp, w.rids_tmp, nullptr, seg_off, w.items, w.n_items, w.counter,
               cfg->small_cap);
  const SegList large{w.large_lo, w.large_hi, nullptr, n_seg};
  if (cfg->large_algo == KPA_SORT_LEARNED)
    return learned_sort_launch(keys_in, rids_in, keys_out, rids_out, large, models, stats, w.lw,
                               st, vals_in, vals_out,
                               cfg->bucket_log2 ? cfg->bucket_log2 : BUCKET_LOG2);
  if (stats) KPA_CHECK(launch_fill_u64(reinterpret_cast<u64*>(stats), STATS_WORDS, 0, st));
  return radix_sort_launch(keys_in, rids_in, keys_out, rids_out, large, w.rw, st,
                           stats_unsupported(stats), vals_in, vals_out);
}

kpa_status check_args(const uint64_t* keys_in, const uint32_t* rids_in, uint64_t* keys_out,
                      uint32_t* rids_out, const uint64_t* seg_off, uint64_t n_cap,
                      const kpa_batch_config* cfg, const kpa_pwl_model* models, void* ws) {
  KPA_CHECK(check_config(cfg));
  KPA_REQUIRE(keys_in && keys_out && rids_out && seg_off && ws, KPA_EINVAL, "null pointer");
  KPA_REQUIRE(keys_in != keys_out && rids_in != (const uint32_t*)rids_out, KPA_EINVAL,
              "inputs must not alias outputs");
  KPA_REQUIRE(aligned(keys_in, 8) && aligned(keys_out, 8) && aligned(rids_in, 4) &&
                  aligned(rids_out, 4) && aligned(seg_off, 8) && aligned(ws, 256),
              KPA_EINVAL, "misaligned pointer");
  KPA_REQUIRE(n_cap < (1ull << 32), KPA_EUNSUPPORTED, "n_cap must be below 2^32");
  KPA_REQUIRE(cfg->large_algo != KPA_SORT_LEARNED || models != nullptr, KPA_EINVAL,
              "learned sort needs models");
  return KPA_OK;
}

// ------------------------------------------------------------ autotuner --

// Signature of a batch for the tuning cache: segment count, capacity and the
// number of segments in each power-of-two size class (4 classes per digit of
// the signature keep it short).
std::string batch_signature(const std::vector<u64>& off, u64 n_cap, u32 algo) {
  u32 cls[8] = {0};
  for (size_t s = 0; s + 1 < off.size(); ++s) {
    const u64 n = off[s + 1] - off[s];
    const int l = n ? 63 - __builtin_clzll(n) : 0;
    cls[std::min(7, l / 4)]++;
  }
  char buf[256];
  std::snprintf(buf, sizeof buf, "n_seg=%zu n_cap_log2=%d algo=%u cls=%u,%u,%u,%u,%u,%u,%u,%u",
                off.size() - 1, n_cap ? 64 - __builtin_clzll(n_cap - 1) : 0, algo, cls[0], cls[1],
                cls[2], cls[3], cls[4], cls[5], cls[6], cls[7]);
  return buf;
}

bool cache_lookup(const char* path, const std::string& sig, kpa_batch_config* cfg, float* ms) {
  if (!path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  while (std::fgets(line, sizeof line, f)) {
    const char* bar = std::strchr(line, '|');
    if (!bar || (size_t)(bar - line) != sig.size() || std::strncmp(line, sig.data(), sig.size()))
      continue;
    kpa_batch_config c{};
    float t = 0;
    c.bucket_log2 = 0;
    if (std::sscanf(bar + 1, " small_cap=%u mid_cap=%u grid=%u large_algo=%u bucket_log2=%u ms=%f",
                    &c.small_cap, &c.mid_cap, &c.grid, &c.large_algo, &c.bucket_log2, &t) == 6 &&
        check_config(&c) == KPA_OK) {
      *cfg = c;  // the last entry for a signature wins
      *ms = t;
      found = true;
    }
  }
  std::fclose(f);
  clear_error();
  return found;
}

void cache_store(const char* path, const std::string& sig, const kpa_batch_config& c, float ms) {
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s| small_cap=%u mid_cap=%u grid=%u large_algo=%u bucket_log2=%u ms=%.4f\n",
               sig.c_str(), c.small_cap, c.mid_cap, c.grid, c.large_algo, c.bucket_log2, ms);
  std::fclose(f);
}

}  // namespace
}  // namespace kpa

using namespace kpa;

extern "C" {

kpa_status kpa_batch_config_default(kpa_sort_algo large_algo, kpa_batch_config* cfg) {
  clear_error();
  KPA_REQUIRE(cfg != nullptr, KPA_EINVAL, "config is null");
  cfg->small_cap = TILE;
  cfg->mid_cap = 1u << 16;
  cfg->grid = 0;
  cfg->large_algo = (uint32_t)large_algo;
  cfg->bucket_log2 = 0;
  return check_config(cfg);
}

kpa_status kpa_batch_sort_workspace_size(uint64_t n_cap, uint32_t n_seg,
                                         const kpa_batch_config* cfg, size_t* bytes) {
  clear_error();
  KPA_REQUIRE(bytes != nullptr, KPA_EINVAL, "bytes is null");
  KPA_CHECK(check_config(cfg));
  Carver c(nullptr);
  BatchWs w;
  KPA_CHECK(batch_plan(n_cap, n_seg ? n_seg : 1, cfg, c, &w));
  *bytes = c.used + 256;
  return KPA_OK;
}

kpa_status kpa_batch_sort(const uint64_t* keys_in, const uint32_t* rids_in, uint64_t* keys_out,
                          uint32_t* rids_out, const uint64_t* seg_off, uint32_t n_seg,
                          uint64_t n_cap, const kpa_batch_config* cfg,
                          const kpa_pwl_model* models, kpa_sort_stats* stats, void* ws,
                          size_t ws_bytes, hipStream_t stream) {
  clear_error();
  KPA_CHECK(check_config(cfg));
  if (n_seg == 0 || n_cap == 0) return KPA_OK;
  KPA_CHECK(check_args(keys_in, rids_in, keys_out, rids_out, seg_off, n_cap, cfg, models, ws));
  Carver c(ws);
  BatchWs w;
  KPA_CHECK(batch_plan(n_cap, n_seg, cfg, c, &w));
  KPA_REQUIRE(c.used <= ws_bytes, KPA_EWORKSPACE, "workspace too small: need %zu bytes", c.used);
  return batch_launch(keys_in, rids_in, keys_out, rids_out, seg_off, n_seg, cfg, models, stats,
                      w, stream);
}

kpa_status kpa_batch_sort_vals_workspace_size(uint64_t n_cap, uint32_t n_seg,
                                              const kpa_batch_config* cfg, size_t* bytes) {
  clear_error();
  KPA_REQUIRE(bytes != nullptr, KPA_EINVAL, "bytes is null");
  KPA_CHECK(check_config(cfg));
  Carver c(nullptr);
  BatchWs w;
  KPA_CHECK(batch_plan(n_cap, n_seg ? n_seg : 1, cfg, c, &w, true));
  *bytes = c.used + 256;
  return KPA_OK;
}

kpa_status kpa_batch_sort_vals(const uint64_t* keys_in, const uint32_t* rids_in,
                               const uint64_t* vals_in, uint64_t* keys_out, uint32_t* rids_out,
                               uint64_t* vals_out, const uint64_t* seg_off, uint32_t n_seg,
                               uint64_t n_cap, const kpa_batch_config* cfg,
                               const kpa_pwl_model* models, kpa_sort_stats* stats, void* ws,
                               size_t ws_bytes, hipStream_t stream) {
  clear_error();
  KPA_CHECK(check_config(cfg));
  if (n_seg == 0 || n_cap == 0) return KPA_OK;
  KPA_CHECK(check_args(keys_in, rids_in, keys_out, rids_out, seg_off, n_cap, cfg, models, ws));
  KPA_REQUIRE(vals_in && vals_out, KPA_EINVAL, "null pointer");
  KPA_REQUIRE(vals_in != vals_out, KPA_EINVAL, "inputs must not alias outputs");
  KPA_REQUIRE(aligned(vals_in, 8) && aligned(vals_out, 8), KPA_EINVAL, "misaligned pointer");
  Carver c(ws);
  BatchWs w;
  KPA_CHECK(batch_plan(n_cap, n_seg, cfg, c, &w, true));
  KPA_REQUIRE(c.used <= ws_bytes, KPA_EWORKSPACE, "workspace too small: need %zu bytes", c.used);
  return batch_launch(keys_in, rids_in, keys_out, rids_out, seg_off, n_seg, cfg, models, stats,
                      w, stream, vals_in, vals_out);
}

kpa_status kpa_batch_autotune(const uint64_t* keys_in, const uint32_t* rids_in,
                              uint64_t* keys_out, uint32_t* rids_out, const uint64_t* seg_off,
                              uint32_t n_seg, uint64_t n_cap, kpa_sort_algo large_algo,
                              const kpa_pwl_model* models, void* ws, size_t ws_bytes,
                              uint32_t reps, const char* cache_path, kpa_batch_config* best,
                              float* best_ms, hipStream_t stream) {
  clear_error();
  KPA_REQUIRE(best != nullptr, KPA_EINVAL, "best is null");
  KPA_CHECK(kpa_batch_config_default(large_algo, best));
  if (best_ms) *best_ms = 0.0f;
  if (n_seg == 0 || n_cap == 0) return KPA_OK;
  KPA_CHECK(check_args(keys_in, rids_in, keys_out, rids_out, seg_off, n_cap, best, models, ws));
  if (reps == 0) reps = 1;
  // The candidates' workspace layouts differ only in the large path, which
  // the caller fixed; size it once.
  size_t need = 0;
  KPA_CHECK(kpa_batch_sort_workspace_size(n_cap, n_seg, best, &need));
  KPA_REQUIRE(need <= ws_bytes, KPA_EWORKSPACE, "workspace too small: need %zu bytes", need);

  std::vector<u64> off(n_seg + 1);
  KPA_HIP(hipMemcpyAsync(off.data(), seg_off, off.size() * sizeof(u64), hipMemcpyDeviceToHost,
                         stream));
  KPA_HIP(hipStreamSynchronize(stream));
  const std::string sig = batch_signature(off, n_cap, (u32)large_algo);
  float cached_ms = 0;
  if (cache_lookup(cache_path, sig, best, &cached_ms)) {
    if (best_ms) *best_ms = cached_ms;
    return KPA_OK;
  }

  std::vector<kpa_batch_config> cand;
  const u32 smalls[] = {1024, 2048, TILE};
  const u32 mids[] = {0, 1u << 14, 1u << 16, 1u << 18};
  for (u32 sc : smalls)
    for (u32 mc : mids) {
      kpa_batch_config c{sc, std::max(sc, mc), 0, (uint32_t)large_algo, 0};
      if (mc != 0 && mc <= sc) continue;
      cand.push_back(c);
    }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  KPA_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    KPA_HIP(hipErrorOutOfMemory);
  }
  float best_t = INFINITY;
  kpa_status rc = KPA_OK;
  // Times one candidate (one warm-up, then `reps` runs) and keeps it if it
  // is the fastest so far.
  auto try_config = [&](const kpa_batch_config& c) {
    rc = kpa_batch_sort(keys_in, rids_in, keys_out, rids_out, seg_off, n_seg, n_cap, &c, models,
                        nullptr, ws, ws_bytes, stream);
    if (rc != KPA_OK) return;
    if (hipEventRecord(e0, stream) != hipSuccess) {
      rc = KPA_EHIP;
      set_error("event record failed in the autotuner");
      return;
    }
    for (u32 r = 0; r < reps && rc == KPA_OK; ++r)
      rc = kpa_batch_sort(keys_in, rids_in, keys_out, rids_out, seg_off, n_seg, n_cap, &c,
                          models, nullptr, ws, ws_bytes, stream);
    if (rc != KPA_OK) return;
    float ms = 0;
    if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      rc = KPA_EHIP;
      set_error("event timing failed in the autotuner");
      return;
    }
    ms /= (float)reps;
    if (ms < best_t) {
      best_t = ms;
      *best = c;
    }
  };
  for (const kpa_batch_config& c : cand) {
    try_config(c);
    if (rc != KPA_OK) break;
  }
  // The learned large path's bucket size, at the best class boundaries (the
  // candidates above ran with the default 2^9).
  if (rc == KPA_OK && large_algo == KPA_SORT_LEARNED) {
    const kpa_batch_config base = *best;
    for (u32 bl : {8u, 10u}) {
      kpa_batch_config c = base;
      c.bucket_log2 = bl;
      try_config(c);
      if (rc != KPA_OK) break;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  KPA_CHECK(rc);
  if (best_ms) *best_ms = best_t;
  cache_store(cache_path, sig, *best, best_t);
  return KPA_OK;
}

}  // extern "C"
