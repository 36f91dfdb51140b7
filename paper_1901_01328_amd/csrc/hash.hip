// Hash GroupBy: the random-access alternative to sort-based grouping that the
// paper's motivation study measures against sorting (Sec. 2.2: an open-
// addressing, pre-allocated table; sort-based grouping was faster on HBM).
//
// An open-addressing table of table_cap slots (a power of two) with linear
// probing, keyed by the SplitMix64 finalizer of the key.  A row claims its
// key's slot with a compare-and-swap on the slot's key (no thread ever waits
// for another), then adds its count and value and raises the maximum with
// atomics.  The all-ones key, which marks free slots, has a slot of its own
// after the table.  Groups come out in table order (not by key), compacted by
// a count, scan and write over 4096-slot tiles.
#include "kpa_internal.hpp"

namespace kpa {

constexpr u64 HASH_FREE = ~0ull;
constexpr u32 HASH_TILE = 4096;

__device__ __forceinline__ u64 hash_mix(u64 z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct HashTab {
  u64* key;  // cap + 1 slots (slot cap: the all-ones key)
  u64* cnt;
  u64* sum;
  u64* mx;
  u32* overflow;
  u64 cap;
};

__global__ void __launch_bounds__(256) k_hash_clear(HashTab t) {
  for (u64 i = (u64)blockIdx.x * 256 + threadIdx.x; i <= t.cap; i += (u64)gridDim.x * 256) {
    t.key[i] = HASH_FREE;
    t.cnt[i] = 0;
    t.sum[i] = 0;
    t.mx[i] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *t.overflow = 0;
}

__global__ void __launch_bounds__(256) k_hash_insert(const unsigned char* __restrict__ rows, u64 n,
                                                     u32 row_bytes, u32 key_off, u32 val_off,
                                                     u32 val_w, HashTab t) {
  const u64 mask = t.cap - 1;
  for (u64 i = (u64)blockIdx.x * 256 + threadIdx.x; i < n; i += (u64)gridDim.x * 256) {
    const unsigned char* r = rows + i * row_bytes;
    const u64 k = *reinterpret_cast<const u64*>(r + key_off);
    const u64 v = val_w == 8 ? *reinterpret_cast<const u64*>(r + val_off)
                             : (u64)*reinterpret_cast<const u32*>(r + val_off);
    u64 slot = t.cap;
    if (k != HASH_FREE) {
      u64 h = hash_mix(k) & mask;
      bool found = false;
      for (u64 probe = 0; probe < t.cap; ++probe) {
        const u64 old = atomicCAS(reinterpret_cast<unsigned long long*>(t.key + h),
                                  (unsigned long long)HASH_FREE, (unsigned long long)k);
        if (old == HASH_FREE || old == k) {
          found = true;
          break;
        }
        h = (h + 1) & mask;
      }
      if (!found) {
        atomicOr(t.overflow, 1u);
        continue;
      }
      slot = h;
    }
    atomicAdd(reinterpret_cast<unsigned long long*>(t.cnt + slot), 1ull);
    atomicAdd(reinterpret_cast<unsigned long long*>(t.sum + slot), (unsigned long long)v);
    atomicMax(reinterpret_cast<unsigned long long*>(t.mx + slot), (unsigned long long)v);
  }
}

// Occupied slots per tile.
__global__ void __launch_bounds__(256) k_hash_tcount(HashTab t, u32* __restrict__ tcount) {
  __shared__ u32 red[WAVES];
  const u64 a = (u64)blockIdx.x * HASH_TILE;
  u32 c = 0;
  for (u64 i = a + threadIdx.x; i < a + HASH_TILE && i <= t.cap; i += 256) c += t.cnt[i] != 0;
  c = wave_sum(c);
  if (__lane_id() == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    u32 s = 0;
    for (int w = 0; w < WAVES; ++w) s += red[w];
    tcount[blockIdx.x] = s;
  }
}

// Exclusive prefix of the tile counts (one workgroup of 1024); the total
// goes to *ngroups (all ones when a key found no slot).
__global__ void __launch_bounds__(1024) k_hash_tscan(u32* __restrict__ tcount, u32 n_tiles,
                                                     const u32* __restrict__ overflow,
                                                     u64* __restrict__ ngroups) {
  __shared__ u32 sm[17];
  u32 carry = 0;
  for (u32 b0 = 0; b0 < n_tiles; b0 += 1024) {
    const u32 b = b0 + threadIdx.x;
    const u32 v = b < n_tiles ? tcount[b] : 0u;
    u32 tot;
    const u32 ex = block_excl_sum<16>(v, sm, &tot);
    if (b < n_tiles) tcount[b] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) *ngroups = *overflow ? ~0ull : (u64)carry;
}

__global__ void __launch_bounds__(256) k_hash_write(HashTab t, const u32* __restrict__ tbase,
                                                    u64 g_cap, u64* __restrict__ gkey,
                                                    u64* __restrict__ gcnt, u64* __restrict__ gsum,
                                                    u64* __restrict__ gmax) {
  __shared__ u32 sc[WAVES + 1];
  const u64 a = (u64)blockIdx.x * HASH_TILE;
  u32 o = tbase[blockIdx.x];
  for (u64 r = 0; r < HASH_TILE; r += 256) {
    const u64 i = a + r + threadIdx.x;
    const bool occ = i <= t.cap && t.cnt[i] != 0;
    u32 tot;
    const u32 ex = block_excl_sum(occ ? 1u : 0u, sc, &tot);
    if (occ && o + ex < g_cap) {
      const u64 g = o + ex;
      gkey[g] = i == t.cap ? HASH_FREE : t.key[i];
      if (gcnt) gcnt[g] = t.cnt[i];
      if (gsum) gsum[g] = t.sum[i];
      if (gmax) gmax[g] = t.mx[i];
    }
    o += tot;
  }
}

struct HashWs {
  HashTab t;
  u32* tcount;
  u32 n_tiles;
};

static void hash_plan(u64 cap, Carver& c, HashWs* w) {
  w->t.cap = cap;
  w->t.key = c.take<u64>(cap + 1);
  w->t.cnt = c.take<u64>(cap + 1);
  w->t.sum = c.take<u64>(cap + 1);
  w->t.mx = c.take<u64>(cap + 1);
  w->t.overflow = c.take<u32>(1);
  w->n_tiles = (u32)ceil_div(cap + 1, HASH_TILE);
  w->tcount = c.take<u32>(w->n_tiles);
}

}  // namespace kpa

using namespace kpa;

extern "C" {

kpa_status kpa_hash_groupby_workspace_size(uint64_t table_cap, size_t* bytes) {
  clear_error();
  KPA_REQUIRE(bytes, KPA_EINVAL, "bytes is null");
  KPA_REQUIRE(table_cap >= 1 && (table_cap & (table_cap - 1)) == 0 && table_cap <= (1ull << 31),
              KPA_EINVAL, "table_cap must be a power of two up to 2^31");
  Carver c(nullptr);
  HashWs w;
  hash_plan(table_cap, c, &w);
  *bytes = c.used + 256;
  return KPA_OK;
}

kpa_status kpa_hash_groupby(const void* rows, uint64_t n, const kpa_row_layout* layout,
                            uint64_t table_cap, uint64_t* out_gkey, uint64_t* out_cnt,
                            uint64_t* out_sum, uint64_t* out_max, uint64_t g_cap,
                            uint64_t* out_ngroups, void* ws, size_t ws_bytes,
                            hipStream_t stream) {
  clear_error();
  KPA_CHECK(check_layout(layout, true, false));
  KPA_REQUIRE(table_cap >= 1 && (table_cap & (table_cap - 1)) == 0 && table_cap <= (1ull << 31),
              KPA_EINVAL, "table_cap must be a power of two up to 2^31");
  KPA_REQUIRE(out_gkey && out_ngroups && ws && (n == 0 || rows), KPA_EINVAL, "null pointer");
  KPA_REQUIRE(aligned(ws, 256) && aligned(out_gkey, 8) && aligned(out_ngroups, 8) &&
                  aligned(out_cnt, 8) && aligned(out_sum, 8) && aligned(out_max, 8) &&
                  (n == 0 || aligned(rows, 16)),
              KPA_EINVAL, "misaligned pointer");
  Carver c(ws);
  HashWs w;
  hash_plan(table_cap, c, &w);
  KPA_REQUIRE(c.used <= ws_bytes, KPA_EWORKSPACE, "workspace too small: need %zu bytes", c.used);
  KPA_LAUNCH("hash_clear", k_hash_clear,
             dim3((u32)std::min<u64>(ceil_div(table_cap + 1, 256), 16384)), dim3(256), 0, stream,
             w.t);
  if (n) {
    KPA_LAUNCH("hash_insert", k_hash_insert, dim3((u32)std::min<u64>(ceil_div(n, 256), 16384)),
               dim3(256), 0, stream, static_cast<const unsigned char*>(rows), n,
               layout->row_bytes, layout->key_off, layout->val_off, layout->val_w, w.t);
  }
  KPA_LAUNCH("hash_compact", k_hash_tcount, dim3(w.n_tiles), dim3(256), 0, stream, w.t, w.tcount);
  KPA_LAUNCH("hash_compact", k_hash_tscan, dim3(1), dim3(1024), 0, stream, w.tcount, w.n_tiles,
             w.t.overflow, out_ngroups);
  KPA_LAUNCH("hash_compact", k_hash_write, dim3(w.n_tiles), dim3(256), 0, stream, w.t, w.tcount,
             g_cap, out_gkey, out_cnt, out_sum, out_max);
  return KPA_OK;
}

}  // extern "C"
