// Library-wide plumbing: errors, argument checks, segment-to-tile mapping,
// fills, and the two pure data-movement primitives (Extract, Materialize).
#include <cstdarg>

#include "kpa_internal.hpp"

namespace kpa {

static thread_local char g_err[512] = "";
static thread_local int g_hip_err = 0;

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  g_hip_err = 0;
}
void set_hip_error(int code) { g_hip_err = code; }
void clear_error() {
  g_err[0] = 0;
  g_hip_err = 0;
}

kpa_status check_layout(const kpa_row_layout* L, bool need_val, bool need_ts) {
  KPA_REQUIRE(L != nullptr, KPA_EINVAL, "layout is null");
  KPA_REQUIRE(L->row_bytes >= 8 && L->row_bytes <= 256 && L->row_bytes % 8 == 0, KPA_EINVAL,
              "row_bytes must be a multiple of 8 in [8, 256]");
  KPA_REQUIRE(L->key_off % 8 == 0 && L->key_off + 8 <= L->row_bytes, KPA_EINVAL,
              "key_off must be 8-aligned and inside the row");
  if (need_val) {
    KPA_REQUIRE((L->val_w == 4 || L->val_w == 8) && L->val_off % L->val_w == 0 &&
                    L->val_off + L->val_w <= L->row_bytes,
                KPA_EINVAL, "bad value column (width 4/8, aligned, inside the row)");
  }
  if (need_ts) {
    KPA_REQUIRE((L->ts_w == 4 || L->ts_w == 8) && L->ts_off % L->ts_w == 0 &&
                    L->ts_off + L->ts_w <= L->row_bytes,
                KPA_EINVAL, "bad timestamp column (width 4/8, aligned, inside the row)");
  }
  return KPA_OK;
}

// One workgroup of 1024 threads scans the per-segment tile counts.
__global__ void __launch_bounds__(1024) k_seg_tiles(const u64* __restrict__ off_a,
                                                    const u64* __restrict__ off_b, u32 n_seg,
                                                    u32 tile, u32* __restrict__ tile_start) {
  __shared__ u32 sm[17];
  const u32 per = (n_seg + 1023) / 1024;
  const u32 s0 = threadIdx.x * per;
  const u32 s1 = min(n_seg, s0 + per);
  u32 local = 0;
  for (u32 s = s0; s < s1; ++s) {
    u64 len = off_a[s + 1] - off_a[s];
    if (off_b) len += off_b[s + 1] - off_b[s];
    u64 t = (len + tile - 1) / tile;
    local += (u32)(t ? t : 1);
  }
  // block exclusive scan over 1024 threads
  u32 incl = wave_incl_sum(local);
  u32 w = threadIdx.x >> 6;
  if (__lane_id() == 63) sm[w] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    u32 acc = 0;
    for (int i = 0; i < 16; ++i) {
      u32 t = sm[i];
      sm[i] = acc;
      acc += t;
    }
    sm[16] = acc;
  }
  __syncthreads();
  u32 run = sm[w] + incl - local;
  for (u32 s = s0; s < s1; ++s) {
    tile_start[s] = run;
    u64 len = off_a[s + 1] - off_a[s];
    if (off_b) len += off_b[s + 1] - off_b[s];
    u64 t = (len + tile - 1) / tile;
    run += (u32)(t ? t : 1);
  }
  if (threadIdx.x == 0) tile_start[n_seg] = sm[16];
}

kpa_status launch_seg_tiles(const u64* off_a, const u64* off_b, u32 n_seg, u32 tile,
                            u32* tile_start, hipStream_t st) {
  KPA_LAUNCH("seg_tiles", k_seg_tiles, dim3(1), dim3(1024), 0, st, off_a, off_b, n_seg, tile,
                     tile_start);
  return KPA_OK;
}

template <class T>
__global__ void __launch_bounds__(256) k_fill(T* __restrict__ p, u64 n, T v) {
  u64 i = (u64)blockIdx.x * 256 + threadIdx.x;
  u64 stride = (u64)gridDim.x * 256;
  for (; i < n; i += stride) p[i] = v;
}

__global__ void __launch_bounds__(BLOCK) k_tile_seg(const u32* __restrict__ tile_start, u32 n_max,
                                                   const u32* __restrict__ n_dev, u64 max_tiles,
                                                   u32* __restrict__ tile_seg) {
  const u32 n_seg = n_dev ? min(*n_dev, n_max) : n_max;
  const u64 total = min<u64>(tile_start[n_seg], max_tiles);
  for (u64 t = (u64)blockIdx.x * BLOCK + threadIdx.x; t < total; t += (u64)gridDim.x * BLOCK)
    tile_seg[t] = find_seg(tile_start, n_seg, (u32)t);
}

kpa_status launch_tile_seg(const u32* tile_start, u32 n_seg, const u32* n_dev, u64 max_tiles,
                           u32* tile_seg, hipStream_t st) {
  KPA_LAUNCH("tile_seg", k_tile_seg, dim3((u32)std::min<u64>(ceil_div(max_tiles, BLOCK), 4096)),
             dim3(BLOCK), 0, st, tile_start, n_seg, n_dev, max_tiles, tile_seg);
  return KPA_OK;
}

kpa_status launch_fill_u32(u32* p, u64 n, u32 v, hipStream_t st) {
  if (n == 0) return KPA_OK;
  u64 blocks = std::min<u64>(ceil_div(n, 256), 8192);
  KPA_LAUNCH("fill", k_fill<u32>, dim3((u32)blocks), dim3(256), 0, st, p, n, v);
  return KPA_OK;
}
kpa_status launch_fill_u64(u64* p, u64 n, u64 v, hipStream_t st) {
  if (n == 0) return KPA_OK;
  u64 blocks = std::min<u64>(ceil_div(n, 256), 8192);
  KPA_LAUNCH("fill", k_fill<u64>, dim3((u32)blocks), dim3(256), 0, st, p, n, v);
  return KPA_OK;
}

// Extract: one thread per row, key copied, rid = base + row (when wanted).
__global__ void __launch_bounds__(256) k_extract(const unsigned char* __restrict__ rows, u64 n,
                                                 u32 row_bytes, u32 key_off, u32 val_off,
                                                 u32 val_w, u32 rid_base, u64* __restrict__ keys,
                                                 u32* __restrict__ rids, u64* __restrict__ vals) {
  u64 i = (u64)blockIdx.x * 256 + threadIdx.x;
  u64 stride = (u64)gridDim.x * 256;
  for (; i < n; i += stride) {
    keys[i] = *reinterpret_cast<const u64*>(rows + i * row_bytes + key_off);
    if (rids) rids[i] = rid_base + (u32)i;
    if (vals) vals[i] = load_val(rows, (u32)i, row_bytes, val_off, val_w);
  }
}

// Materialize: rows are copied in 8-byte words; a wave covers consecutive
// output words, so writes are coalesced and each source row is read whole.
__global__ void __launch_bounds__(256) k_materialize(const u32* __restrict__ rids, u64 n,
                                                     const u64* __restrict__ rows, u32 words,
                                                     u64* __restrict__ out) {
  u64 total = n * words;
  u64 i = (u64)blockIdx.x * 256 + threadIdx.x;
  u64 stride = (u64)gridDim.x * 256;
  for (; i < total; i += stride) {
    u64 r = i / words;
    u32 w = (u32)(i - r * words);
    out[i] = rows[(u64)rids[r] * words + w];
  }
}

// Specialisation for 32-byte rows: two 16-byte loads and stores per row.
__global__ void __launch_bounds__(256) k_materialize32(const u32* __restrict__ rids, u64 n,
                                                       const uint4* __restrict__ rows,
                                                       uint4* __restrict__ out) {
  u64 total = n * 2;
  u64 i = (u64)blockIdx.x * 256 + threadIdx.x;
  u64 stride = (u64)gridDim.x * 256;
  for (; i < total; i += stride) {
    u64 r = i >> 1;
    out[i] = rows[(u64)rids[r] * 2 + (i & 1)];
  }
}

}  // namespace kpa

using namespace kpa;

extern "C" {

int32_t kpa_version(void) { return 10000; }

const char* kpa_last_error_string(void) { return kpa::g_err; }

int32_t kpa_last_hip_error(void) { return kpa::g_hip_err; }

kpa_status kpa_device_check(int32_t* out) {
  KPA_REQUIRE(out != nullptr, KPA_EINVAL, "out is null");
  int dev = 0;
  KPA_HIP(hipGetDevice(&dev));
  hipDeviceProp_t p;
  KPA_HIP(hipGetDeviceProperties(&p, dev));
  *out = (std::strncmp(p.gcnArchName, "gfx950", 6) == 0) ? 1 : 0;
  return KPA_OK;
}

kpa_status kpa_extract(const void* rows, uint64_t n, const kpa_row_layout* layout,
                       uint32_t rid_base, uint64_t* out_keys, uint32_t* out_rids,
                       uint64_t* out_vals, hipStream_t stream) {
  clear_error();
  KPA_CHECK(check_layout(layout, out_vals != nullptr, false));
  if (n == 0) return KPA_OK;
  KPA_REQUIRE(rows && out_keys, KPA_EINVAL, "null pointer");
  KPA_REQUIRE(aligned(rows, 16) && aligned(out_keys, 8) && aligned(out_rids, 4) &&
                  aligned(out_vals, 8),
              KPA_EINVAL, "misaligned pointer");
  KPA_REQUIRE(n + rid_base <= (1ull << 32), KPA_EUNSUPPORTED, "rids exceed 32 bits");
  u64 blocks = std::min<u64>(ceil_div(n, 256), 16384);
  KPA_LAUNCH("extract", k_extract, dim3((u32)blocks), dim3(256), 0, stream,
             static_cast<const unsigned char*>(rows), n, layout->row_bytes, layout->key_off,
             layout->val_off, layout->val_w, rid_base, out_keys, out_rids, out_vals);
  return KPA_OK;
}

kpa_status kpa_materialize(const uint32_t* rids, uint64_t n, const void* rows, uint32_t row_bytes,
                           void* out_rows, hipStream_t stream) {
  clear_error();
  if (n == 0) return KPA_OK;
  KPA_REQUIRE(rids && rows && out_rows, KPA_EINVAL, "null pointer");
  KPA_REQUIRE(row_bytes >= 8 && row_bytes <= 256 && row_bytes % 8 == 0, KPA_EINVAL,
              "row_bytes must be a multiple of 8 in [8, 256]");
  KPA_REQUIRE(aligned(rows, 16) && aligned(out_rows, 16) && aligned(rids, 4), KPA_EINVAL,
              "misaligned pointer");
  if (row_bytes == 32) {
    u64 blocks = std::min<u64>(ceil_div(n * 2, 256), 32768);
    KPA_LAUNCH("materialize", k_materialize32, dim3((u32)blocks), dim3(256), 0, stream, rids, n,
               static_cast<const uint4*>(rows), static_cast<uint4*>(out_rows));
  } else {
    u32 words = row_bytes / 8;
    u64 blocks = std::min<u64>(ceil_div(n * words, 256), 32768);
    KPA_LAUNCH("materialize", k_materialize, dim3((u32)blocks), dim3(256), 0, stream, rids, n,
               static_cast<const u64*>(rows), words, static_cast<u64*>(out_rows));
  }
  
  return KPA_OK;
}

}  // extern "C"
