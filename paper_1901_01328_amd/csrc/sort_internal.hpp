// Workspace layouts and launch entry points shared between the sort files.
#pragma once

#include "kpa_internal.hpp"

namespace kpa {

constexpr u32 SEG_UNSUPPORTED = 1u << 31;

struct RadixWs {
  u64* keys_tmp;
  u32* rids_tmp;
  u32* hist;        // n_seg * 8 * 256: digit counts, then exclusive offsets
  u32* seg_mask;    // n_seg: bit p set when pass p is needed
  u32* tile_start;  // n_seg + 1
  u32* status0;     // look-back words, max_tiles * 256, two alternating buffers
  u32* status1;
  u32* counters;    // 16 tile counters (one per pass)
  u64 max_tiles;
};

kpa_status radix_sort_plan(u64 n_cap, u32 n_seg, Carver& c, RadixWs* w);
kpa_status radix_sort_launch(const u64* keys_in, const u32* rids_in, u64* keys_out,
                             u32* rids_out, const u64* seg_off, u32 n_seg, const RadixWs& w,
                             hipStream_t st);

}  // namespace kpa
