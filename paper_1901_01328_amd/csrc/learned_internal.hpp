// Workspace layout and launch entry of the learned-splitter sort.
#pragma once

#include "sort_internal.hpp"

namespace kpa {

struct LearnedWs {
  u64 placeholder;
};

kpa_status learned_sort_plan(u64 n_cap, u32 n_seg, Carver& c, LearnedWs* w);
kpa_status learned_sort_launch(const u64* keys_in, const u32* rids_in, u64* keys_out,
                               u32* rids_out, const u64* seg_off, u32 n_seg, u64 n_cap,
                               const kpa_pwl_model* models, kpa_sort_stats* stats,
                               const RadixWs& rw, const LearnedWs& lw, hipStream_t st);

}  // namespace kpa
