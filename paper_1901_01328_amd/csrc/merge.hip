// Merge (Table 2: two sorted KPAs -> one sorted KPA, sequential access).
//
// Merge path (Green, McColl & Bader, 2012): output position d of the merge is
// reached after taking i entries of A and d - i of B, where i is found by a
// binary search along the cross diagonal.  One kernel computes the split at
// every 4096-entry output tile boundary; a second loads each tile's A and B
// ranges into LDS, lets each thread find its own 16-output split inside them
// and merge sequentially, then writes the tile out coalesced.  Stable: on
// equal keys A's entries come first.
#include <vector>

#include "kpa_internal.hpp"

namespace kpa {

// Number of A entries among the first d outputs (ties taken from A first).
__device__ __forceinline__ u64 merge_split(const u64* a, u64 na, const u64* b, u64 nb, u64 d) {
  u64 lo = d > nb ? d - nb : 0, hi = d < na ? d : na;
  while (lo < hi) {
    const u64 mid = (lo + hi) >> 1;
    if (a[mid] <= b[d - mid - 1]) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__global__ void __launch_bounds__(BLOCK) k_merge_splits(const u64* __restrict__ a, u64 na,
                                                        const u64* __restrict__ b, u64 nb,
                                                        u64 n_tiles, u64* __restrict__ split) {
  const u64 t = (u64)blockIdx.x * BLOCK + threadIdx.x;
  if (t > n_tiles) return;
  const u64 d = min(t * (u64)TILE, na + nb);
  split[t] = merge_split(a, na, b, nb, d);
}

struct MergeSmem {
  u64 k[TILE];
  u32 r[TILE];
};

// Output tile t (entries [t*TILE, min((t+1)*TILE, na+nb)) of the merge of A
// and B) from the splits at its two ends, split[0] and split[1].
__device__ __forceinline__ void merge_tile(MergeSmem& sm, const u64* __restrict__ ak,
                                           const u32* __restrict__ ar, u64 na,
                                           const u64* __restrict__ bk,
                                           const u32* __restrict__ br, u64 nb,
                                           const u64* __restrict__ split, u64 t,
                                           u64* __restrict__ ok, u32* __restrict__ orr) {
  const u64 d0 = t * TILE, d1 = min(d0 + TILE, na + nb);
  const u64 i0 = split[0], i1 = split[1];
  const u64 j0 = d0 - i0, j1 = d1 - i1;
  const u32 la = (u32)(i1 - i0), lb = (u32)(j1 - j0);
  // A part at [0, la), B part at [la, la + lb)
  for (u32 x = threadIdx.x; x < la; x += BLOCK) {
    sm.k[x] = ak[i0 + x];
    sm.r[x] = ar[i0 + x];
  }
  for (u32 x = threadIdx.x; x < lb; x += BLOCK) {
    sm.k[la + x] = bk[j0 + x];
    sm.r[la + x] = br[j0 + x];
  }
  __syncthreads();
  const u64* A = sm.k;
  const u64* B = sm.k + la;
  const u32 dd = min((u32)threadIdx.x * ITEMS, la + lb);
  u32 lo = dd > lb ? dd - lb : 0, hi = dd < la ? dd : la;
  while (lo < hi) {
    const u32 mid = (lo + hi) >> 1;
    if (A[mid] <= B[dd - mid - 1]) lo = mid + 1; else hi = mid;
  }
  u32 ia = lo, ib = dd - lo;
  u64 outk[ITEMS];
  u32 outr[ITEMS];
#pragma unroll
  for (int q = 0; q < ITEMS; ++q) {
    const bool takea = ib >= lb || (ia < la && A[ia] <= B[ib]);
    const u32 src = takea ? ia : la + ib;
    outk[q] = src < la + lb ? sm.k[src] : 0ull;
    outr[q] = src < la + lb ? sm.r[src] : 0u;
    ia += takea;
    ib += !takea;
  }
  __syncthreads();
  const u32 n = (u32)(d1 - d0);
#pragma unroll
  for (int q = 0; q < ITEMS; ++q) {
    const u32 o = threadIdx.x * ITEMS + q;
    if (o < n) {
      sm.k[o] = outk[q];
      sm.r[o] = outr[q];
    }
  }
  __syncthreads();
  for (u32 x = threadIdx.x; x < n; x += BLOCK) {
    ok[d0 + x] = sm.k[x];
    orr[d0 + x] = sm.r[x];
  }
}

__global__ void __launch_bounds__(BLOCK) k_merge_tiles(const u64* __restrict__ ak,
                                                       const u32* __restrict__ ar, u64 na,
                                                       const u64* __restrict__ bk,
                                                       const u32* __restrict__ br, u64 nb,
                                                       const u64* __restrict__ split,
                                                       u64* __restrict__ ok, u32* __restrict__ orr) {
  __shared__ MergeSmem sm;
  merge_tile(sm, ak, ar, na, bk, br, nb, split + blockIdx.x, blockIdx.x, ok, orr);
}

// One round of the pairwise merge of many runs, all pairs in one launch.
// Pair q merges A = src[a0, a1) and B = src[a1, b1) into dst[a0, b1) (b1 = a1
// for an unpaired last run, which is copied); t0 = output tiles of the pairs
// before it.  The round's split array holds, pair after pair, the splits at
// each of a pair's tiles + 1 boundaries: pair q's start at t0 + q.
struct MergePair {
  u64 a0, a1, b1, t0;
};
constexpr u32 PAIR_CHUNK = 64;  // descriptors copied per launch (2 KiB of arguments)
struct PairChunk {
  MergePair p[PAIR_CHUNK];
};
// Pairs planned per call on the device path; more nonempty runs take the
// per-pair launches.
constexpr u32 MR_PLAN_RUNS = 1024;
constexpr u64 MR_PLAN_DESC = MR_PLAN_RUNS + 64;  // all rounds' pairs (< runs + rounds)

__global__ void __launch_bounds__(PAIR_CHUNK) k_merge_desc(PairChunk c, u32 cnt,
                                                           MergePair* __restrict__ out) {
  if (threadIdx.x < cnt) out[threadIdx.x] = c.p[threadIdx.x];
}

// Largest q < n_pairs with key(q) <= x, key nondecreasing in q and key(0) = 0.
template <typename KeyOf>
__device__ __forceinline__ u32 last_le(u32 n_pairs, u64 x, KeyOf key) {
  u32 lo = 0, hi = n_pairs - 1;
  while (lo < hi) {
    const u32 mid = (lo + hi + 1) >> 1;
    if (key(mid) <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ void __launch_bounds__(BLOCK) k_merge_round_splits(const u64* __restrict__ src,
                                                              const MergePair* __restrict__ pr,
                                                              u32 n_pairs, u64 n_bounds,
                                                              u64* __restrict__ split) {
  const u64 g = (u64)blockIdx.x * BLOCK + threadIdx.x;
  if (g >= n_bounds) return;
  const u32 q = last_le(n_pairs, g, [&](u32 i) { return pr[i].t0 + i; });
  const MergePair p = pr[q];
  const u64 na = p.a1 - p.a0, nb = p.b1 - p.a1;
  const u64 d = min((g - p.t0 - q) * (u64)TILE, na + nb);
  split[g] = merge_split(src + p.a0, na, src + p.a1, nb, d);
}

__global__ void __launch_bounds__(BLOCK) k_merge_round_tiles(const u64* __restrict__ sk,
                                                             const u32* __restrict__ sr,
                                                             const MergePair* __restrict__ pr,
                                                             u32 n_pairs,
                                                             const u64* __restrict__ split,
                                                             u64* __restrict__ dk,
                                                             u32* __restrict__ dr) {
  __shared__ MergeSmem sm;
  const u64 b = blockIdx.x;
  const u32 q = last_le(n_pairs, b, [&](u32 i) { return pr[i].t0; });
  const MergePair p = pr[q];
  merge_tile(sm, sk + p.a0, sr + p.a0, p.a1 - p.a0, sk + p.a1, sr + p.a1, p.b1 - p.a1,
             split + p.t0 + q + (b - p.t0), b - p.t0, dk + p.a0, dr + p.a0);
}

__global__ void __launch_bounds__(BLOCK) k_copy_kpa(const u64* __restrict__ k, const u32* __restrict__ r,
                                                    u64 n, u64* __restrict__ ok,
                                                    u32* __restrict__ orr) {
  for (u64 i = (u64)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (u64)gridDim.x * BLOCK) {
    ok[i] = k[i];
    orr[i] = r[i];
  }
}

kpa_status merge_launch(const u64* ak, const u32* ar, u64 na, const u64* bk, const u32* br, u64 nb,
                        u64* ok, u32* orr, u64* split, hipStream_t st) {
  const u64 n = na + nb;
  if (n == 0) return KPA_OK;
  const u64 tiles = ceil_div(n, TILE);
  KPA_LAUNCH("merge_splits", k_merge_splits, dim3((u32)ceil_div(tiles + 1, BLOCK)), dim3(BLOCK), 0,
             st, ak, na, bk, nb, tiles, split);
  KPA_LAUNCH("merge_tiles", k_merge_tiles, dim3((u32)tiles), dim3(BLOCK), 0, st, ak, ar, na, bk, br,
             nb, split, ok, orr);
  return KPA_OK;
}

}  // namespace kpa

using namespace kpa;

extern "C" {

kpa_status kpa_merge_workspace_size(uint64_t na, uint64_t nb, size_t* bytes) {
  clear_error();
  KPA_REQUIRE(bytes, KPA_EINVAL, "bytes is null");
  *bytes = (ceil_div(na + nb, TILE) + 2) * sizeof(u64) + 256;
  return KPA_OK;
}

kpa_status kpa_merge(const uint64_t* a_keys, const uint32_t* a_rids, uint64_t na,
                     const uint64_t* b_keys, const uint32_t* b_rids, uint64_t nb,
                     uint64_t* out_keys, uint32_t* out_rids, void* ws, size_t ws_bytes,
                     hipStream_t stream) {
  clear_error();
  if (na + nb == 0) return KPA_OK;
  KPA_REQUIRE((na == 0 || (a_keys && a_rids)) && (nb == 0 || (b_keys && b_rids)) && out_keys &&
                  out_rids && ws,
              KPA_EINVAL, "null pointer");
  KPA_REQUIRE(aligned(ws, 8) && aligned(out_keys, 8) && aligned(out_rids, 4) &&
                  (na == 0 || (aligned(a_keys, 8) && aligned(a_rids, 4))) &&
                  (nb == 0 || (aligned(b_keys, 8) && aligned(b_rids, 4))),
              KPA_EINVAL, "misaligned pointer");
  KPA_REQUIRE(out_keys != a_keys && out_keys != b_keys, KPA_EINVAL, "outputs alias inputs");
  size_t need = 0;
  kpa_merge_workspace_size(na, nb, &need);
  KPA_REQUIRE(ws_bytes >= need, KPA_EWORKSPACE, "workspace too small: need %zu bytes", need);
  return merge_launch(a_keys, a_rids, na, b_keys, b_rids, nb, out_keys, out_rids,
                      static_cast<u64*>(ws), stream);
}

kpa_status kpa_merge_runs_workspace_size(uint64_t n, size_t* bytes) {
  clear_error();
  KPA_REQUIRE(bytes, KPA_EINVAL, "bytes is null");
  Carver c(nullptr);
  c.take<u64>(n);
  c.take<u32>(n);
  c.take<u64>(ceil_div(n, TILE) + 2 + 2 * (u64)MR_PLAN_RUNS);
  c.take<MergePair>(MR_PLAN_DESC);
  *bytes = c.used + 256;
  return KPA_OK;
}

// Pairwise rounds: runs 2k and 2k+1 merge into run k of the next round (an
// unpaired last run is carried over), alternating between the caller's arrays
// and a workspace copy; the last round writes the output.  Empty runs are
// dropped first.  Up to MR_PLAN_RUNS runs, every round is one split launch
// and one tile launch over all of its pairs, whose descriptors are planned on
// the host and copied into the workspace by kernel arguments (so the call
// holds no host-to-device copy and can be captured); beyond that, each pair
// is merged by its own launches.
kpa_status kpa_merge_runs(uint64_t* keys, uint32_t* rids, const uint64_t* run_off, uint32_t n_runs,
                          uint64_t* out_keys, uint32_t* out_rids, void* ws, size_t ws_bytes,
                          hipStream_t stream) {
  clear_error();
  KPA_REQUIRE(run_off != nullptr, KPA_EINVAL, "run_off is null");
  if (n_runs == 0) return KPA_OK;
  const u64 n = run_off[n_runs] - run_off[0];
  for (u32 r = 0; r < n_runs; ++r)
    KPA_REQUIRE(run_off[r + 1] >= run_off[r], KPA_EINVAL, "run offsets decrease");
  if (n == 0) return KPA_OK;
  KPA_REQUIRE(keys && rids && out_keys && out_rids && ws, KPA_EINVAL, "null pointer");
  KPA_REQUIRE(aligned(ws, 256), KPA_EINVAL, "misaligned workspace");
  size_t need = 0;
  kpa_merge_runs_workspace_size(n, &need);
  KPA_REQUIRE(ws_bytes >= need, KPA_EWORKSPACE, "workspace too small: need %zu bytes", need);
  Carver c(ws);
  u64* tk = c.take<u64>(n);
  u32* tr = c.take<u32>(n);
  u64* split = c.take<u64>(ceil_div(n, TILE) + 2 + 2 * (u64)MR_PLAN_RUNS);
  MergePair* desc = c.take<MergePair>(MR_PLAN_DESC);
  const u64 base = run_off[0];
  std::vector<u64> off{0};
  for (u32 r = 0; r < n_runs; ++r)
    if (run_off[r + 1] > run_off[r]) off.push_back(run_off[r + 1] - base);
  u64* ck = keys + base;
  u32* cr = rids + base;
  if (off.size() == 2) {
    KPA_LAUNCH("copy_kpa", k_copy_kpa, dim3((u32)std::min<u64>(ceil_div(n, BLOCK), 8192)),
               dim3(BLOCK), 0, stream, ck, cr, n, out_keys, out_rids);
    return KPA_OK;
  }
  const bool planned = off.size() - 1 <= MR_PLAN_RUNS;
  // Rounds on the host: each round's pairs and its output tiles.
  struct Round {
    u64 first, pairs, tiles;
  };
  std::vector<MergePair> pairs;
  std::vector<Round> rounds;
  for (std::vector<u64> o = off; o.size() > 2;) {
    const size_t runs = o.size() - 1;
    Round rd{pairs.size(), 0, 0};
    std::vector<u64> next{0};
    for (size_t p = 0; p < runs; p += 2) {
      const u64 b1 = p + 1 < runs ? o[p + 2] : o[p + 1];
      pairs.push_back(MergePair{o[p], o[p + 1], b1, rd.tiles});
      rd.tiles += ceil_div(b1 - o[p], TILE);
      next.push_back(b1);
    }
    rd.pairs = pairs.size() - rd.first;
    rounds.push_back(rd);
    o.swap(next);
  }
  if (planned) {
    for (size_t i = 0; i < pairs.size(); i += PAIR_CHUNK) {
      PairChunk chunk;
      const u32 cnt = (u32)std::min<size_t>(PAIR_CHUNK, pairs.size() - i);
      for (u32 j = 0; j < cnt; ++j) chunk.p[j] = pairs[i + j];
      KPA_LAUNCH("merge_desc", k_merge_desc, dim3(1), dim3(PAIR_CHUNK), 0, stream, chunk, cnt,
                 desc + i);
    }
  }
  // buffers: current source, and the next destination
  u64* src_k = ck;
  u32* src_r = cr;
  bool src_is_ws = false;
  for (size_t ri = 0; ri < rounds.size(); ++ri) {
    const Round& rd = rounds[ri];
    const bool last = ri + 1 == rounds.size();
    u64* dst_k = last ? out_keys : (src_is_ws ? ck : tk);
    u32* dst_r = last ? out_rids : (src_is_ws ? cr : tr);
    if (planned) {
      const u64 bounds = rd.tiles + rd.pairs;
      KPA_LAUNCH("merge_splits", k_merge_round_splits, dim3((u32)ceil_div(bounds, BLOCK)),
                 dim3(BLOCK), 0, stream, src_k, desc + rd.first, (u32)rd.pairs, bounds, split);
      KPA_LAUNCH("merge_tiles", k_merge_round_tiles, dim3((u32)rd.tiles), dim3(BLOCK), 0, stream,
                 src_k, src_r, desc + rd.first, (u32)rd.pairs, split, dst_k, dst_r);
    } else {
      for (u64 q = rd.first; q < rd.first + rd.pairs; ++q) {
        const MergePair& p = pairs[q];
        KPA_CHECK(merge_launch(src_k + p.a0, src_r + p.a0, p.a1 - p.a0, src_k + p.a1,
                               src_r + p.a1, p.b1 - p.a1, dst_k + p.a0, dst_r + p.a0, split,
                               stream));
      }
    }
    src_k = dst_k;
    src_r = dst_r;
    src_is_ws = !src_is_ws;
  }
  return KPA_OK;
}

}  // extern "C"
