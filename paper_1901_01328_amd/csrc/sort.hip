// Public entry points of Sort (Table 2).  Radix path in radix.hip, learned
// path in learned.hip.
#include "sort_internal.hpp"
#include "learned_internal.hpp"

using namespace kpa;

namespace {

kpa_status sort_plan(u64 n_cap, u32 n_seg, kpa_sort_algo algo, Carver& c, RadixWs* rw,
                     LearnedWs* lw, bool vals = false) {
  if (algo == KPA_SORT_LEARNED) return learned_sort_plan(n_cap, n_seg, c, lw, vals);
  return radix_sort_plan(n_cap, n_seg, c, rw, vals);
}

__global__ void k_one_segment(u64* seg_off, u64 n) {
  seg_off[0] = 0;
  seg_off[1] = n;
}

}  // namespace

extern "C" {

kpa_status kpa_sort_workspace_size(uint64_t n_cap, uint32_t n_seg, kpa_sort_algo algo,
                                   size_t* bytes) {
  clear_error();
  KPA_REQUIRE(bytes != nullptr, KPA_EINVAL, "bytes is null");
  KPA_REQUIRE(algo == KPA_SORT_RADIX || algo == KPA_SORT_LEARNED, KPA_EINVAL, "bad algo");
  Carver c(nullptr);
  c.take<u64>(2);  // single-segment offsets for kpa_sort
  RadixWs rw;
  LearnedWs lw;
  KPA_CHECK(sort_plan(n_cap, n_seg ? n_seg : 1, algo, c, &rw, &lw));
  *bytes = c.used + 256;
  return KPA_OK;
}

}  // extern "C"

namespace {

kpa_status sort_segmented(const uint64_t* keys_in, const uint32_t* rids_in, const u64* vals_in,
                          uint64_t* keys_out, uint32_t* rids_out, u64* vals_out,
                          const uint64_t* seg_off, uint32_t n_seg, uint64_t n_cap,
                          kpa_sort_algo algo, const kpa_pwl_model* models, kpa_sort_stats* stats,
                          void* ws, size_t ws_bytes, hipStream_t stream) {
  const bool vals = vals_in != nullptr;
  KPA_REQUIRE(algo == KPA_SORT_RADIX || algo == KPA_SORT_LEARNED, KPA_EINVAL, "bad algo");
  if (n_seg == 0 || n_cap == 0) return KPA_OK;
  KPA_REQUIRE(keys_in && keys_out && rids_out && seg_off && ws, KPA_EINVAL, "null pointer");
  KPA_REQUIRE(keys_in != keys_out && rids_in != (const uint32_t*)rids_out, KPA_EINVAL,
              "inputs must not alias outputs");
  KPA_REQUIRE(aligned(keys_in, 8) && aligned(keys_out, 8) && aligned(rids_in, 4) &&
                  aligned(rids_out, 4) && aligned(seg_off, 8) && aligned(ws, 256),
              KPA_EINVAL, "misaligned pointer");
  KPA_REQUIRE(n_cap < (1ull << 32), KPA_EUNSUPPORTED, "n_cap must be below 2^32");
  KPA_REQUIRE(algo != KPA_SORT_LEARNED || models != nullptr, KPA_EINVAL,
              "learned sort needs models");
  Carver c(ws);
  c.take<u64>(2);
  RadixWs rw;
  LearnedWs lw;
  KPA_CHECK(sort_plan(n_cap, n_seg, algo, c, &rw, &lw, vals));
  KPA_REQUIRE(c.used <= ws_bytes, KPA_EWORKSPACE, "workspace too small: need %zu bytes",
              c.used);
  if (algo == KPA_SORT_RADIX) {
    if (stats) KPA_CHECK(launch_fill_u64(reinterpret_cast<u64*>(stats), STATS_WORDS, 0, stream));
    KPA_CHECK(radix_sort_launch(keys_in, rids_in, keys_out, rids_out,
                                seg_list_from_offsets(seg_off, n_seg), rw, stream,
                                stats_unsupported(stats), vals_in, vals_out));
  } else {
    KPA_CHECK(learned_sort_launch(keys_in, rids_in, keys_out, rids_out,
                                  seg_list_from_offsets(seg_off, n_seg), models, stats, lw,
                                  stream, vals_in, vals_out));
  }
  return KPA_OK;
}

}  // namespace

extern "C" {

kpa_status kpa_sort_segmented(const uint64_t* keys_in, const uint32_t* rids_in,
                              uint64_t* keys_out, uint32_t* rids_out, const uint64_t* seg_off,
                              uint32_t n_seg, uint64_t n_cap, kpa_sort_algo algo,
                              const kpa_pwl_model* models, kpa_sort_stats* stats, void* ws,
                              size_t ws_bytes, hipStream_t stream) {
  clear_error();
  return sort_segmented(keys_in, rids_in, nullptr, keys_out, rids_out, nullptr, seg_off, n_seg,
                        n_cap, algo, models, stats, ws, ws_bytes, stream);
}

kpa_status kpa_sort_vals_workspace_size(uint64_t n_cap, uint32_t n_seg, kpa_sort_algo algo,
                                        size_t* bytes) {
  clear_error();
  KPA_REQUIRE(bytes != nullptr, KPA_EINVAL, "bytes is null");
  KPA_REQUIRE(algo == KPA_SORT_RADIX || algo == KPA_SORT_LEARNED, KPA_EINVAL, "bad algo");
  Carver c(nullptr);
  c.take<u64>(2);
  RadixWs rw;
  LearnedWs lw;
  KPA_CHECK(sort_plan(n_cap, n_seg ? n_seg : 1, algo, c, &rw, &lw, true));
  *bytes = c.used + 256;
  return KPA_OK;
}

kpa_status kpa_sort_segmented_vals(const uint64_t* keys_in, const uint32_t* rids_in,
                                   const uint64_t* vals_in, uint64_t* keys_out,
                                   uint32_t* rids_out, uint64_t* vals_out,
                                   const uint64_t* seg_off, uint32_t n_seg, uint64_t n_cap,
                                   kpa_sort_algo algo, const kpa_pwl_model* models,
                                   kpa_sort_stats* stats, void* ws, size_t ws_bytes,
                                   hipStream_t stream) {
  clear_error();
  if (n_seg == 0 || n_cap == 0) return KPA_OK;
  KPA_REQUIRE(vals_in && vals_out, KPA_EINVAL, "null pointer");
  KPA_REQUIRE(vals_in != vals_out, KPA_EINVAL, "inputs must not alias outputs");
  KPA_REQUIRE(aligned(vals_in, 8) && aligned(vals_out, 8), KPA_EINVAL, "misaligned pointer");
  return sort_segmented(keys_in, rids_in, vals_in, keys_out, rids_out, vals_out, seg_off, n_seg,
                        n_cap, algo, models, stats, ws, ws_bytes, stream);
}

kpa_status kpa_sort(const uint64_t* keys_in, const uint32_t* rids_in, uint64_t n,
                    uint64_t* keys_out, uint32_t* rids_out, kpa_sort_algo algo,
                    const kpa_pwl_model* model, kpa_sort_stats* stats, void* ws, size_t ws_bytes,
                    hipStream_t stream) {
  clear_error();
  if (n == 0) return KPA_OK;
  KPA_REQUIRE(ws && aligned(ws, 256), KPA_EINVAL, "workspace null or misaligned");
  KPA_REQUIRE(n < MAX_SEG_ENTRIES, KPA_EUNSUPPORTED, "a segment must hold fewer than 2^30 keys");
  u64* off = reinterpret_cast<u64*>(ws);  // first 16 bytes of the workspace
  KPA_LAUNCH("one_segment", k_one_segment, dim3(1), dim3(1), 0, stream, off, (u64)n);
  return kpa_sort_segmented(keys_in, rids_in, keys_out, rids_out, off, 1, n, algo, model, stats,
                            ws, ws_bytes, stream);
}

}  // extern "C"
