// Internal helpers shared by the kernels of libkpa (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/kpa.h"

typedef uint64_t u64;
typedef uint32_t u32;
typedef int64_t i64;

namespace kpa {

// ----------------------------------------------------------------- errors --
void set_error(const char* fmt, ...);
void clear_error();
void set_hip_error(int code);  // the HIP error behind the next KPA_EHIP

#define KPA_REQUIRE(cond, code, ...) \
  do {                               \
    if (!(cond)) {                   \
      ::kpa::set_error(__VA_ARGS__); \
      return (code);                 \
    }                                \
  } while (0)

#define KPA_HIP(call)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) {                                                            \
      ::kpa::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                       __LINE__);                                                      \
      ::kpa::set_hip_error((int)e_);                                                   \
      return KPA_EHIP;                                                                 \
    }                                                                                  \
  } while (0)

#define KPA_LAUNCHED()                                                                       \
  do {                                                                                       \
    hipError_t e_ = hipGetLastError();                                                       \
    if (e_ != hipSuccess) {                                                                  \
      ::kpa::set_error("kernel launch failed: %s (%s:%d)", hipGetErrorString(e_), __FILE__, \
                       __LINE__);                                                            \
      ::kpa::set_hip_error((int)e_);                                                         \
      return KPA_EHIP;                                                                       \
    }                                                                                        \
  } while (0)

bool prof_enabled();
int prof_begin(const char* name, hipStream_t st);
void prof_end(int slot, hipStream_t st);

// Launch a kernel, timed by the profiler when it is enabled.
#define KPA_LAUNCH(name, kernel, grid, block, shmem, st, ...)         \
  do {                                                               \
    int slot_ = ::kpa::prof_begin(name, st);                         \
    hipLaunchKernelGGL(kernel, grid, block, shmem, st, __VA_ARGS__); \
    ::kpa::prof_end(slot_, st);                                      \
    KPA_LAUNCHED();                                                  \
  } while (0)

#define KPA_CHECK(expr)            \
  do {                             \
    kpa_status s_ = (expr);        \
    if (s_ != KPA_OK) return s_;   \
  } while (0)

inline bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

kpa_status check_layout(const kpa_row_layout* L, bool need_val, bool need_ts);

// -------------------------------------------------------------- workspace --
// Carves 256-byte aligned sub-buffers out of one caller workspace.  With a
// null base it only measures.
struct Carver {
  char* base;
  size_t used = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <class T>
  T* take(size_t count) {
    size_t off = (used + 255) & ~size_t(255);
    used = off + count * sizeof(T) + 0;
    return base ? reinterpret_cast<T*>(base + off) : nullptr;
  }
};

// ------------------------------------------------------------- constants --
constexpr int BLOCK = 256;           // threads per workgroup (4 waves of 64)
constexpr int WAVES = BLOCK / 64;
#ifndef KPA_ITEMS
#define KPA_ITEMS 16
#endif
constexpr int ITEMS = KPA_ITEMS;     // entries per thread in a tile
constexpr int TILE = BLOCK * ITEMS;  // 4096 entries per tile
constexpr u32 ST_AGG = 1u << 30;     // look-back word: tile aggregate ready
constexpr u32 ST_PRE = 2u << 30;     // look-back word: inclusive prefix ready
constexpr u32 ST_VAL = (1u << 30) - 1;
constexpr u64 MAX_SEG_ENTRIES = 1ull << 30;

inline u64 ceil_div(u64 a, u64 b) { return (a + b - 1) / b; }
inline u64 max_tiles(u64 n_cap, u32 n_seg, u64 tile) { return ceil_div(n_cap, tile) + n_seg + 1; }

// Shared launches (common.hip).
// tile_start[s] = sum over s' < s of max(1, ceil(len(s')/tile)), len from one or
// the sum of two offset arrays; tile_start[n_seg] = total.
kpa_status launch_seg_tiles(const u64* off_a, const u64* off_b, u32 n_seg, u32 tile,
                            u32* tile_start, hipStream_t st);
kpa_status launch_fill_u32(u32* p, u64 n, u32 v, hipStream_t st);
// tile_seg[t] = segment of tile t for every tile of a tile map (tile_start,
// n_seg + 1 entries), so that per-tile kernels look their segment up with one
// load instead of a binary search.  tile_seg holds max_tiles entries.
// When n_dev is given the map has *n_dev (at most n_seg) segments.
kpa_status launch_tile_seg(const u32* tile_start, u32 n_seg, const u32* n_dev, u64 max_tiles,
                           u32* tile_seg, hipStream_t st);
kpa_status launch_fill_u64(u64* p, u64 n, u64 v, hipStream_t st);

}  // namespace kpa

// ============================================================ device side ==
#ifdef __HIPCC__
namespace kpa {

__device__ __forceinline__ u32 lane_id() { return __lane_id(); }
__device__ __forceinline__ u64 lanemask_lt() {
  u32 l = __lane_id();
  return (l == 0) ? 0ull : (~0ull >> (64 - l));
}
__device__ __forceinline__ u64 ballot(bool p) { return __ballot(p); }

// Relaxed agent-scope atomic access to look-back words (coherent across XCDs).
__device__ __forceinline__ u32 ld_status(const u32* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_status(u32* p, u32 v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Segment lookup: largest s with tile_start[s] <= t (tile_start nondecreasing).
__device__ __forceinline__ u32 find_seg(const u32* tile_start, u32 n_seg, u32 t) {
  u32 lo = 0, hi = n_seg;  // answer in [lo, hi)
  while (hi - lo > 1) {
    u32 mid = (lo + hi) >> 1;
    if (tile_start[mid] <= t) lo = mid; else hi = mid;
  }
  return lo;
}

// The first active lane's value of a u32, in a scalar register.  The builtin
// returns int; it is converted back here so that widening the result never
// sign-extends (a 64-bit index assembled from two halves stays unsigned).
__device__ __forceinline__ u32 first_lane(u32 v) { return (u32)__builtin_amdgcn_readfirstlane(v); }

// DPP lane moves (GFX9 encodings): row_shr:n shifts within rows of 16
// lanes, row_bcast:15 / row_bcast:31 broadcast lane 15 / 31 of the rows
// below into the rows that row_mask selects, wave_shr:1 shifts the whole
// wave by one lane.  Lanes without a source (or outside row_mask) keep `old`.
// A DPP move reads another lane's register directly, with no trip through
// LDS as a shuffle takes.
constexpr int DPP_ROW_SHR = 0x110, DPP_BCAST15 = 0x142, DPP_BCAST31 = 0x143, DPP_WAVE_SHR1 = 0x138;

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ u32 dpp32(u32 old, u32 v) {
  return (u32)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROW_MASK, 0xF, false);
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ u64 dpp64(u64 old, u64 v) {
  const u32 lo = dpp32<CTRL, ROW_MASK>((u32)old, (u32)v);
  const u32 hi = dpp32<CTRL, ROW_MASK>((u32)(old >> 32), (u32)(v >> 32));
  return ((u64)hi << 32) | lo;
}
template <int CTRL, int ROW_MASK, class T>
__device__ __forceinline__ T dpp_move(T old, T v) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit lanes");
  if constexpr (sizeof(T) == 8)
    return (T)dpp64<CTRL, ROW_MASK>((u64)old, (u64)v);
  else
    return (T)dpp32<CTRL, ROW_MASK>((u32)old, (u32)v);
}

// Inclusive scan over the wave (Hillis-Steele within rows of 16 lanes, then
// the two row broadcasts): lane l gets op over lanes 0..l, op(earlier, later)
// associative with identity e.  Every lane of the wave must be active.
template <class T, class Op>
__device__ __forceinline__ T wave_incl_scan(T v, T e, Op op) {
  v = op(dpp_move<DPP_ROW_SHR + 1, 0xF>(e, v), v);
  v = op(dpp_move<DPP_ROW_SHR + 2, 0xF>(e, v), v);
  v = op(dpp_move<DPP_ROW_SHR + 4, 0xF>(e, v), v);
  v = op(dpp_move<DPP_ROW_SHR + 8, 0xF>(e, v), v);
  v = op(dpp_move<DPP_BCAST15, 0xA>(e, v), v);
  v = op(dpp_move<DPP_BCAST31, 0xC>(e, v), v);
  return v;
}

// Lane 63's value, the same in every lane (a scalar read).
template <class T>
__device__ __forceinline__ T lane63(T v) {
  if constexpr (sizeof(T) == 8) {
    const u32 lo = (u32)__builtin_amdgcn_readlane((int)(u32)(u64)v, 63);
    const u32 hi = (u32)__builtin_amdgcn_readlane((int)(u32)((u64)v >> 32), 63);
    return (T)(((u64)hi << 32) | lo);
  } else {
    return (T)(u32)__builtin_amdgcn_readlane((int)(u32)v, 63);
  }
}

// op over the whole wave, in every lane.  Every lane must be active.
template <class T, class Op>
__device__ __forceinline__ T wave_reduce(T v, T e, Op op) {
  return lane63(wave_incl_scan(v, e, op));
}

// Wave-wide inclusive sum of u32.
__device__ __forceinline__ u32 wave_incl_sum(u32 v) {
  return wave_incl_scan(v, 0u, [](u32 a, u32 b) { return a + b; });
}

// Block-wide exclusive sum of one u32 per thread (NW waves of 64 threads);
// returns the exclusive prefix and writes the block total to *total.  Uses
// `sm` (NW+1 u32).
template <int NW = WAVES>
__device__ __forceinline__ u32 block_excl_sum(u32 v, u32* sm, u32* total) {
  u32 incl = wave_incl_sum(v);
  u32 w = threadIdx.x >> 6;
  if (__lane_id() == 63) sm[w] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    u32 acc = 0;
    for (int i = 0; i < NW; ++i) {
      u32 t = sm[i];
      sm[i] = acc;
      acc += t;
    }
    sm[NW] = acc;
  }
  __syncthreads();
  u32 r = sm[w] + incl - v;
  *total = sm[NW];
  __syncthreads();
  return r;
}

template <class T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    T t = __shfl_xor(v, o, 64);
    v = t > v ? t : v;
  }
  return v;
}
template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ u64 load_val(const unsigned char* rows, u32 rid, u32 row_bytes,
                                        u32 val_off, u32 val_w) {
  const unsigned char* p = rows + (u64)rid * row_bytes + val_off;
  return val_w == 8 ? *reinterpret_cast<const u64*>(p) : (u64)*reinterpret_cast<const u32*>(p);
}

}  // namespace kpa
#endif
