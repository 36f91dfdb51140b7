// KPA maintenance primitives of pipeline execution (Sec. 4.3):
//  * KeySwap (Table 2): load a nonresident column through the pointers and
//    make it the resident key;
//  * in-place update of the resident keys from a key-value table held in
//    device memory (the external join of the paper's pipeline example), and
//    write-back of the resident keys to their rows' column, so that later
//    KeySwap and Materialize see the new values;
//  * Materialize coalesced with Extract: the rows are emitted in KPA order
//    and, while each row is in registers, the next operator's KPA is
//    extracted from it.
#include "kpa_internal.hpp"

namespace kpa {

__global__ void __launch_bounds__(256) k_keyswap(const u32* __restrict__ rids, u64 n,
                                                 const unsigned char* __restrict__ rows,
                                                 u32 row_bytes, u32 col_off, u32 col_w,
                                                 u64* __restrict__ out_keys) {
  for (u64 i = (u64)blockIdx.x * 256 + threadIdx.x; i < n; i += (u64)gridDim.x * 256)
    out_keys[i] = load_val(rows, rids[i], row_bytes, col_off, col_w);
}

constexpr u32 KU_LDS = 2048;  // tables up to this size are searched in LDS

// Lower bound of x among t[0..n) (ascending): first index with t[i] >= x.
__device__ __forceinline__ u64 lower_bound_u64(const u64* t, u64 n, u64 x) {
  u64 lo = 0, hi = n;
  while (lo < hi) {
    const u64 mid = (lo + hi) >> 1;
    if (t[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__global__ void __launch_bounds__(256) k_key_update(u64* __restrict__ keys, u64 n,
                                                    const u64* __restrict__ tkeys,
                                                    const u64* __restrict__ tvals, u64 tn,
                                                    u64* __restrict__ missing) {
  __shared__ u64 sk[KU_LDS], sv[KU_LDS];
  const bool in_lds = tn <= KU_LDS;
  if (in_lds) {
    for (u32 j = threadIdx.x; j < tn; j += 256) {
      sk[j] = tkeys[j];
      sv[j] = tvals[j];
    }
    __syncthreads();
  }
  const u64* tk = in_lds ? sk : tkeys;
  const u64* tv = in_lds ? sv : tvals;
  u32 miss = 0;
  for (u64 i = (u64)blockIdx.x * 256 + threadIdx.x; i < n; i += (u64)gridDim.x * 256) {
    const u64 x = keys[i];
    const u64 j = lower_bound_u64(tk, tn, x);
    if (j < tn && tk[j] == x) keys[i] = tv[j];
    else ++miss;
  }
  miss = wave_sum(miss);
  if (__lane_id() == 0 && miss) atomicAdd(reinterpret_cast<unsigned long long*>(missing), (u64)miss);
}

__global__ void __launch_bounds__(256) k_key_writeback(const u64* __restrict__ keys,
                                                       const u32* __restrict__ rids, u64 n,
                                                       unsigned char* __restrict__ rows,
                                                       u32 row_bytes, u32 col_off) {
  for (u64 i = (u64)blockIdx.x * 256 + threadIdx.x; i < n; i += (u64)gridDim.x * 256)
    *reinterpret_cast<u64*>(rows + (u64)rids[i] * row_bytes + col_off) = keys[i];
}

// 32-byte rows: two lanes per row, 16 bytes each; the lane holding the new
// key's half writes it to the KPA.
__global__ void __launch_bounds__(256) k_mat_extract32(const u32* __restrict__ rids, u64 n,
                                                       const uint4* __restrict__ rows,
                                                       u32 key_off, u32 rid_base,
                                                       uint4* __restrict__ out_rows,
                                                       u64* __restrict__ out_keys,
                                                       u32* __restrict__ out_rids) {
  const u64 total = n * 2;
  for (u64 i = (u64)blockIdx.x * 256 + threadIdx.x; i < total; i += (u64)gridDim.x * 256) {
    const u64 r = i >> 1;
    const u32 half = (u32)(i & 1);
    const uint4 v = rows[(u64)rids[r] * 2 + half];
    out_rows[i] = v;
    if ((key_off >> 4) == half) {
      const bool hi = (key_off & 8) != 0;
      out_keys[r] = hi ? ((u64)v.w << 32 | v.z) : ((u64)v.y << 32 | v.x);
      out_rids[r] = rid_base + (u32)r;
    }
  }
}

// Any row size: one thread per 8-byte word of the output.
__global__ void __launch_bounds__(256) k_mat_extract(const u32* __restrict__ rids, u64 n,
                                                     const u64* __restrict__ rows, u32 words,
                                                     u32 key_word, u32 rid_base,
                                                     u64* __restrict__ out_rows,
                                                     u64* __restrict__ out_keys,
                                                     u32* __restrict__ out_rids) {
  const u64 total = n * words;
  for (u64 i = (u64)blockIdx.x * 256 + threadIdx.x; i < total; i += (u64)gridDim.x * 256) {
    const u64 r = i / words;
    const u32 wd = (u32)(i - r * words);
    const u64 v = rows[(u64)rids[r] * words + wd];
    out_rows[i] = v;
    if (wd == key_word) {
      out_keys[r] = v;
      out_rids[r] = rid_base + (u32)r;
    }
  }
}

}  // namespace kpa

using namespace kpa;

extern "C" {

kpa_status kpa_keyswap(const uint32_t* rids, uint64_t n, const void* rows, uint32_t row_bytes,
                       uint32_t col_off, uint32_t col_w, uint64_t* out_keys, hipStream_t stream) {
  clear_error();
  KPA_REQUIRE(row_bytes >= 8 && row_bytes <= 256 && row_bytes % 8 == 0, KPA_EINVAL,
              "row_bytes must be a multiple of 8 in [8, 256]");
  KPA_REQUIRE((col_w == 4 || col_w == 8) && col_off % col_w == 0 && col_off + col_w <= row_bytes,
              KPA_EINVAL, "bad column (width 4/8, aligned, inside the row)");
  if (n == 0) return KPA_OK;
  KPA_REQUIRE(rids && rows && out_keys, KPA_EINVAL, "null pointer");
  KPA_REQUIRE(aligned(rids, 4) && aligned(rows, 16) && aligned(out_keys, 8), KPA_EINVAL,
              "misaligned pointer");
  const u64 blocks = std::min<u64>(ceil_div(n, 256), 16384);
  KPA_LAUNCH("keyswap", k_keyswap, dim3((u32)blocks), dim3(256), 0, stream, rids, n,
             static_cast<const unsigned char*>(rows), row_bytes, col_off, col_w, out_keys);
  return KPA_OK;
}

kpa_status kpa_key_update(uint64_t* keys, uint64_t n, const uint64_t* table_keys,
                          const uint64_t* table_vals, uint64_t table_n, uint64_t* out_missing,
                          hipStream_t stream) {
  clear_error();
  KPA_REQUIRE(out_missing && aligned(out_missing, 8), KPA_EINVAL, "out_missing null or misaligned");
  KPA_CHECK(launch_fill_u64(out_missing, 1, 0, stream));
  if (n == 0) return KPA_OK;
  KPA_REQUIRE(keys && (table_n == 0 || (table_keys && table_vals)), KPA_EINVAL, "null pointer");
  KPA_REQUIRE(aligned(keys, 8) && aligned(table_keys, 8) && aligned(table_vals, 8), KPA_EINVAL,
              "misaligned pointer");
  const u64 blocks = std::min<u64>(ceil_div(n, 256), 8192);
  KPA_LAUNCH("key_update", k_key_update, dim3((u32)blocks), dim3(256), 0, stream, keys, n,
             table_keys, table_vals, table_n, out_missing);
  return KPA_OK;
}

kpa_status kpa_key_writeback(const uint64_t* keys, const uint32_t* rids, uint64_t n, void* rows,
                             uint32_t row_bytes, uint32_t col_off, hipStream_t stream) {
  clear_error();
  KPA_REQUIRE(row_bytes >= 8 && row_bytes <= 256 && row_bytes % 8 == 0, KPA_EINVAL,
              "row_bytes must be a multiple of 8 in [8, 256]");
  KPA_REQUIRE(col_off % 8 == 0 && col_off + 8 <= row_bytes, KPA_EINVAL,
              "col_off must be 8-aligned and inside the row");
  if (n == 0) return KPA_OK;
  KPA_REQUIRE(keys && rids && rows, KPA_EINVAL, "null pointer");
  KPA_REQUIRE(aligned(keys, 8) && aligned(rids, 4) && aligned(rows, 16), KPA_EINVAL,
              "misaligned pointer");
  const u64 blocks = std::min<u64>(ceil_div(n, 256), 16384);
  KPA_LAUNCH("key_writeback", k_key_writeback, dim3((u32)blocks), dim3(256), 0, stream, keys, rids,
             n, static_cast<unsigned char*>(rows), row_bytes, col_off);
  return KPA_OK;
}

kpa_status kpa_materialize_extract(const uint32_t* rids, uint64_t n, const void* rows,
                                   uint32_t row_bytes, uint32_t key_off, uint32_t rid_base,
                                   void* out_rows, uint64_t* out_keys, uint32_t* out_rids,
                                   hipStream_t stream) {
  clear_error();
  KPA_REQUIRE(row_bytes >= 8 && row_bytes <= 256 && row_bytes % 8 == 0, KPA_EINVAL,
              "row_bytes must be a multiple of 8 in [8, 256]");
  KPA_REQUIRE(key_off % 8 == 0 && key_off + 8 <= row_bytes, KPA_EINVAL,
              "key_off must be 8-aligned and inside the row");
  if (n == 0) return KPA_OK;
  KPA_REQUIRE(rids && rows && out_rows && out_keys && out_rids, KPA_EINVAL, "null pointer");
  KPA_REQUIRE(aligned(rids, 4) && aligned(rows, 16) && aligned(out_rows, 16) &&
                  aligned(out_keys, 8) && aligned(out_rids, 4),
              KPA_EINVAL, "misaligned pointer");
  KPA_REQUIRE(n + rid_base <= (1ull << 32), KPA_EUNSUPPORTED, "rids exceed 32 bits");
  if (row_bytes == 32) {
    const u64 blocks = std::min<u64>(ceil_div(n * 2, 256), 32768);
    KPA_LAUNCH("materialize_extract", k_mat_extract32, dim3((u32)blocks), dim3(256), 0, stream,
               rids, n, static_cast<const uint4*>(rows), key_off, rid_base,
               static_cast<uint4*>(out_rows), out_keys, out_rids);
  } else {
    const u32 words = row_bytes / 8;
    const u64 blocks = std::min<u64>(ceil_div(n * words, 256), 32768);
    KPA_LAUNCH("materialize_extract", k_mat_extract, dim3((u32)blocks), dim3(256), 0, stream,
               rids, n, static_cast<const u64*>(rows), words, key_off / 8, rid_base,
               static_cast<u64*>(out_rows), out_keys, out_rids);
  }
  return KPA_OK;
}

}  // extern "C"
