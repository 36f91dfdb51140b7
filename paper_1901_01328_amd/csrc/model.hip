// CDF models for the learned-splitter sort: the piecewise-linear fit.
//
// For a segment of n sorted keys, kmin/kmax are its first and last keys and
// knot j (0..S) is the fraction of keys strictly below the boundary
// kmin + floor(j*(kmax-kmin)/S), computed as an exact count by binary search
// and rounded once (double quotient, then float).
#include "kpa_internal.hpp"

namespace kpa {

__global__ void __launch_bounds__(BLOCK) k_pwl_fit(const u64* __restrict__ keys,
                                                   const u64* __restrict__ seg_off, u32 n_seg,
                                                   u32 S, kpa_pwl_model* __restrict__ out) {
  for (u32 s = blockIdx.x; s < n_seg; s += gridDim.x) {
    const u64 a = seg_off[s], b = seg_off[s + 1];
    const u64 n = b - a;
    kpa_pwl_model& M = out[s];
    if (n == 0) {
      if (threadIdx.x == 0) {
        M.kmin = M.kmax = 0;
        M.n_seg = 0;
        M.reserved = 0;
      }
      continue;
    }
    const u64 kmin = keys[a], kmax = keys[b - 1];
    const u64 span = kmax - kmin;
    const u64 q = span / S, r = span % S;
    for (u32 j = threadIdx.x; j <= S; j += BLOCK) {
      const u64 bound = kmin + (u64)j * q + ((u64)j * r) / S;
      u64 lo = 0, hi = n;  // first index with key >= bound
      while (lo < hi) {
        const u64 mid = (lo + hi) >> 1;
        if (keys[a + mid] < bound) lo = mid + 1; else hi = mid;
      }
      M.knots[j] = (float)((double)lo / (double)n);
    }
    if (threadIdx.x == 0) {
      M.kmin = kmin;
      M.kmax = kmax;
      M.n_seg = S;
      M.reserved = 0;
    }
  }
}

}  // namespace kpa

using namespace kpa;

extern "C" {

kpa_status kpa_pwl_fit(const uint64_t* sorted_keys, const uint64_t* seg_off, uint32_t n_seg,
                       uint32_t n_seg_model, kpa_pwl_model* out_models, hipStream_t stream) {
  clear_error();
  KPA_REQUIRE(n_seg_model >= 1 && n_seg_model <= KPA_PWL_MAX_SEG, KPA_EUNSUPPORTED,
              "n_seg_model must be in [1, %d]", KPA_PWL_MAX_SEG);
  if (n_seg == 0) return KPA_OK;
  KPA_REQUIRE(sorted_keys && seg_off && out_models, KPA_EINVAL, "null pointer");
  KPA_REQUIRE(aligned(sorted_keys, 8) && aligned(seg_off, 8) && aligned(out_models, 8),
              KPA_EINVAL, "misaligned pointer");
  KPA_LAUNCH("pwl_fit", k_pwl_fit, dim3(std::min<u32>(n_seg, 4096)), dim3(BLOCK), 0, stream,
             sorted_keys, seg_off, n_seg, n_seg_model, out_models);
  return KPA_OK;
}

}  // extern "C"
