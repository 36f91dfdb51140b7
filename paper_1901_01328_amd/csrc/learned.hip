// Learned-splitter sort.
//
// A monotone model F (kpa_pwl_model: piecewise-linear CDF fitted on the sorted
// KPA of an earlier window) maps each key to a bucket b = floor(B*F(key)),
// B = 2^bits chosen per segment so that buckets hold about 512 entries.
// F is applied over the segment's key range, taken from a sample of its keys.
// Because F never decreases, every key of bucket b precedes every key of
// bucket b+1, so the sort reduces to
//   1. a stable scatter by bucket id: one onesweep pass for up to 8 bits of
//      bucket id, else two with the bits split evenly (digit_sort.hpp with
//      the model as digit function);
//   2. a finishing pass: the 2048-entry stretches of the output in which a
//      bucket starts are listed, and a workgroup per listed stretch sorts the
//      buckets that start in it (at most 4096 entries) in LDS: by a refined
//      bucket id (8 more bits of F), then by key within runs of one refined
//      id, with a byte-wise LSD radix as the fallback;
//   3. oversize chunks (a bucket larger than the on-chip capacity, typically
//      a heavy key plus a few light keys the model could not separate) are
//      listed.  Each is split stably three ways around its most frequent key
//      (a sample's mode): the equal part is final (one key, input order), the
//      parts below and above are sorted on chip when small enough, else split
//      again; after two rounds what remains goes to the radix path.
// A segment whose model fails validation (knots not finite, outside [0, 1],
// or decreasing) gets a single bucket and so goes to the radix path whole.
// The output equals the radix sort's byte for byte: both are the stable sort.
#include "digit_sort.hpp"
#include "learned_internal.hpp"
#include "onchip_sort.hpp"

namespace kpa {

struct LearnedDF {
  static constexpr int PASSES = 2;
  static constexpr int SMEM = KPA_PWL_MAX_SEG + 1;  // floats of LDS for the knots
  struct Params {
    const SegModel* segm;
    const kpa_pwl_model* models;  // segment s's knots: models[s].knots
  };
  // A segment's model and knots held in registers by a scatter workgroup: the
  // loads are issued while the previous tile is written, and the knots go to
  // LDS when the segment's tile starts.  Every knot of the array is read, so
  // no load waits for the model.
  static constexpr int KNOT_REGS = (KPA_PWL_MAX_SEG + 1 + PASS_THREADS - 1) / PASS_THREADS;
  struct Staged {
    SegModel m;
    float k[KNOT_REGS];
  };
  SegModel m;
  const lds_float* kn;
  LearnedDF() = default;
  __device__ __forceinline__ LearnedDF(const Params& p, u32 seg) : m(p.segm[seg]) {}
  __device__ __forceinline__ explicit LearnedDF(const Staged& s) : m(s.m) {}
  static __device__ __forceinline__ Staged fetch(const Params& p, u32 seg) {
    Staged s;
    s.m = p.segm[seg];
    const float* g = p.models[seg].knots;
#pragma unroll
    for (int i = 0; i < KNOT_REGS; ++i) {
      const u32 j = threadIdx.x + (u32)i * PASS_THREADS;
      s.k[i] = j <= (u32)KPA_PWL_MAX_SEG ? g[j] : 0.0f;
    }
    return s;
  }
  // All threads of a scatter workgroup; the caller synchronizes.
  __device__ __forceinline__ void bind_staged(const Staged& s, float* lds) {
#pragma unroll
    for (int i = 0; i < KNOT_REGS; ++i) {
      const u32 j = threadIdx.x + (u32)i * PASS_THREADS;
      if (j <= (u32)KPA_PWL_MAX_SEG) lds[j] = s.k[i];
    }
    kn = (const lds_float*)lds;
  }
  // All threads: copy the knots to LDS and evaluate from there (the caller
  // synchronizes before the first use).
  __device__ __forceinline__ void bind(float* sm) { kn = bind_knots(m, sm); }
  // A bucket id of more than 8 bits is split evenly over the two passes (13
  // bits: 7 + 6 rather than 8 + 5).  Bucket ids are spread evenly by design,
  // so a pass's digit runs in a tile get longer, and its writes more
  // contiguous, with fewer digit values.
  __device__ __forceinline__ u32 lo_bits() const { return m.bits <= 8 ? 8u : (m.bits + 1) / 2; }
  __device__ __forceinline__ u32 digit(u64 k, u32 pass) const {
    const u32 b = model_bucket(m, kn, k), lb = lo_bits();
    return pass == 0 ? (b & ((1u << lb) - 1)) : (b >> lb);
  }
  __device__ __forceinline__ void digits(u64 k, u32 (&d)[PASSES]) const {
    const u32 b = model_bucket(m, kn, k), lb = lo_bits();
    d[0] = b & ((1u << lb) - 1);
    d[1] = b >> lb;
  }
};

enum StatIdx { ST_BUCKETS = 0, ST_ONCHIP, ST_EQUAL, ST_FB_ENTRIES, ST_FB_BUCKETS, ST_VIOL };

__device__ __forceinline__ void stat_add(kpa_sort_stats* st, int idx, u64 v) {
  if (st && v) atomicAdd(reinterpret_cast<unsigned long long*>(st) + idx, (unsigned long long)v);
}

// Key range of every segment, estimated from a sample: the first BLOCK keys
// of each of its TILE-entry tiles (one key in 16).  Only the model's
// resolution depends on it: keys outside the estimate get F = 0 or 1 and land
// in the first or last bucket, where they belong.  Each workgroup takes a
// contiguous run of tiles and keeps SAMPLE_TILES tiles' loads in flight per
// thread; it publishes a segment's extremes (one atomic pair) when the
// segment changes and at the end.
constexpr int SAMPLE_TILES = 16;

__global__ void __launch_bounds__(BLOCK) k_seg_minmax(const u64* __restrict__ keys, SegList sl,
                                                      const u32* __restrict__ tile_start,
                                                      const u32* __restrict__ tile_seg,
                                                      u64* __restrict__ kmin,
                                                      u64* __restrict__ kmax) {
  __shared__ u64 red[2 * WAVES];
  const u32 n_seg = sl.n();
  const u32 total = tile_start[n_seg];
  const u32 per = (total + gridDim.x - 1) / gridDim.x;
  const u32 t0 = blockIdx.x * per, t1 = min(total, t0 + per);
  u64 lo = ~0ull, hi = 0;
  u32 cur = NONE;
  auto publish = [&]() {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const u64 l2 = __shfl_xor(lo, o, 64), h2 = __shfl_xor(hi, o, 64);
      lo = l2 < lo ? l2 : lo;
      hi = h2 > hi ? h2 : hi;
    }
    __syncthreads();
    if (__lane_id() == 0) {
      red[threadIdx.x >> 6] = lo;
      red[WAVES + (threadIdx.x >> 6)] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 0; w < WAVES; ++w) {
        lo = red[w] < lo ? red[w] : lo;
        hi = red[WAVES + w] > hi ? red[WAVES + w] : hi;
      }
      if (lo <= hi) {  // the segment had keys in these tiles
        atomicMin(reinterpret_cast<unsigned long long*>(kmin + cur), (unsigned long long)lo);
        atomicMax(reinterpret_cast<unsigned long long*>(kmax + cur), (unsigned long long)hi);
      }
    }
    lo = ~0ull;
    hi = 0;
  };
  for (u32 tg = t0; tg < t1; tg += SAMPLE_TILES) {
    u32 sg[SAMPLE_TILES];
    u64 k[SAMPLE_TILES];
    bool v[SAMPLE_TILES];
#pragma unroll
    for (int j = 0; j < SAMPLE_TILES; ++j) {
      const u32 t = tg + j;
      sg[j] = t < t1 ? tile_seg[t] : NONE;
      v[j] = false;
      k[j] = 0;
      if (t < t1) {
        const u32 s = sg[j];
        const u64 i = sl.lo[s] + (u64)(t - tile_start[s]) * TILE + threadIdx.x;
        v[j] = i < sl.hi[s];
        if (v[j]) k[j] = keys[i];
      }
    }
#pragma unroll
    for (int j = 0; j < SAMPLE_TILES; ++j) {
      if (sg[j] == NONE) break;
      if (sg[j] != cur) {
        if (cur != NONE) publish();
        cur = sg[j];
      }
      if (v[j]) {
        lo = k[j] < lo ? k[j] : lo;
        hi = k[j] > hi ? k[j] : hi;
      }
    }
  }
  if (cur != NONE) publish();
}

// The model's knots describe the shape of the CDF over the key range it was
// fitted on; it is applied over the segment's own range [kmin, kmax] (taken
// from the keys), so that a window whose keys moved by an offset since the
// model's window keeps the model's resolution.
__global__ void __launch_bounds__(BLOCK) k_learned_setup(const kpa_pwl_model* __restrict__ models,
                                                         SegList sl,
                                                         const u64* __restrict__ cur_min,
                                                         const u64* __restrict__ cur_max,
                                                         SegModel* __restrict__ segm,
                                                         kpa_sort_stats* stats, u32 bucket_log2) {
  const u32 n_seg = sl.n();
  for (u32 s = blockIdx.x; s < n_seg; s += gridDim.x) {
    const kpa_pwl_model& M = models[s];
    const u64 n = sl.hi[s] - sl.lo[s];
    const u32 nseg = M.n_seg;
    bool ok = nseg >= 1 && nseg <= KPA_PWL_MAX_SEG && M.kmax >= M.kmin && n > 0;
    if (ok) {
      for (u32 j = threadIdx.x; j <= nseg; j += BLOCK) {
        const float a = M.knots[j];
        bool good = a >= 0.0f && a <= 1.0f;  // false for NaN
        if (j > 0) good = good && a >= M.knots[j - 1];
        ok = ok && good;
      }
    }
    ok = __syncthreads_and(ok);
    if (threadIdx.x == 0) {
      SegModel m;
      m.kmin = ok ? cur_min[s] : M.kmin;
      m.kmax = ok ? cur_max[s] : M.kmax;
      m.nseg = ok ? nseg : 1;
      const u64 span = m.kmax - m.kmin;
      u32 sh = 0;
      while ((span >> sh) > 0xFFFFFFFFull) ++sh;
      m.sh = sh;
      m.hspan = (u32)(span >> sh);
      m.scale = (ok && m.hspan) ? (float)nseg / (float)m.hspan : 0.0f;
      m.valid = ok ? 1u : 0u;
      m.knots = M.knots;
      // A segment too large for the look-back words keeps one bucket: it goes
      // to the pivot rounds and the radix path whole (which copies what stays
      // too large through and counts it).
      u32 bits = 0;
      if (ok && n > FCAP && n < MAX_SEG_ENTRIES) {
        const u64 want = (n + (1ull << bucket_log2) - 1) >> bucket_log2;
        while (bits < MAX_BUCKET_BITS && (1ull << bits) < want) ++bits;
      }
      m.bits = bits;
      segm[s] = m;
      if (n) {
        stat_add(stats, ST_BUCKETS, 1ull << bits);
        if (!ok) stat_add(stats, ST_VIOL, 1);
      }
    }
    __syncthreads();
  }
}

// The finishing workgroup: 8 waves, two workgroups per CU (LDS-bound), so
// that each SIMD keeps four waves to hide LDS and memory latency.
constexpr int FIN_WAVES = 8;
constexpr u32 FIN_THREADS = FIN_WAVES * 64;
constexpr int FIN_ITEMS = FCAP / FIN_THREADS;  // entries per thread of a full chunk
constexpr u32 SHORT_RUN = 64;  // runs up to this length are ranked by counting
constexpr u32 LONG_RUNS = 64;  // long runs a chunk may split before the byte-wise sort

template <int NW>
struct FinishSmemT {
  static constexpr int kWaves = NW;
  u32 whist[NW][RADIX];
  u32 lstart[RADIX];
  u32 scan[NW + 1];
  u32 red[NW];
  u32 red_inv[NW];
  u64 red64[2 * NW];
  float knots[KPA_PWL_MAX_SEG + 1];
  u64 skeys[FCAP + 1];
  u32 srids[FCAP];
  u32 srel[FCAP + 1];  // refined bucket id (relative to the chunk's first bucket)
  u32 flag;
  u32 n_long;                // long runs with inversions still to split
  u32 long_lo[LONG_RUNS];
  u32 long_hi[LONG_RUNS];
};
using FinishSmem = FinishSmemT<FIN_WAVES>;

// Stable ranks of the entries of a short stretch [s, e) of sm by (key,
// position): each of the first e-s threads counts the entries that precede
// its own, then all move at once.  e - s <= FIN_THREADS.
__device__ __forceinline__ void rank_short(FinishSmem& sm, u32 s, u32 e) {
  const u32 tid = threadIdx.x;
  u64 k = 0;
  u32 r = 0, dst = 0;
  const bool mine = tid < e - s;
  if (mine) {
    const u32 i = s + tid;
    k = sm.skeys[i];
    r = sm.srids[i];
    u32 rank = 0;
    for (u32 q = s; q < e; ++q) {
      const u64 kq = sm.skeys[q];
      rank += (kq < k) || (kq == k && q < i);
    }
    dst = s + rank;
  }
  __syncthreads();
  if (mine) {
    sm.skeys[dst] = k;
    sm.srids[dst] = r;
  }
  __syncthreads();
}

// Sorts the registered long runs (runs of one refined id longer than
// SHORT_RUN that are out of key order; typically a frequent key next to a
// few others).  Each run is split stably three ways around the most frequent
// of 64 evenly spaced sample keys: the equal part is final, a part of at
// most SHORT_RUN entries is ranked by counting, a longer one is split again.
// When more than LONG_RUNS runs or parts need splitting the chunk is left to
// the byte-wise sort (sm.flag).
__device__ void split_long_runs(FinishSmem& sm) {
  const u32 tid = threadIdx.x;
  const u32 lane = __lane_id();
  __syncthreads();
  for (u32 head = 0;; ++head) {
    const u32 n_long = min(sm.n_long, LONG_RUNS);
    if (head >= n_long || sm.flag) break;
    const u32 s = sm.long_lo[head], e = sm.long_hi[head];
    const u32 len = e - s;
    // pivot: the mode of 64 evenly spaced keys (wave 0)
    if (tid < 64) {
      const u64 kv = sm.skeys[s + (u32)(((u64)lane * len) / 64)];
      u32 c = 0;
      for (int q = 0; q < 64; ++q) c += __shfl(kv, q, 64) == kv;
      u32 best = (c << 6) | (63u - lane);
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const u32 t = __shfl_xor(best, o, 64);
        best = t > best ? t : best;
      }
      const u64 piv = __shfl(kv, 63 - (int)(best & 63u), 64);
      if (lane == 0) sm.red64[0] = piv;
    }
    __syncthreads();
    const u64 piv = sm.red64[0];
    // each thread owns a contiguous part of the run (at most FIN_ITEMS entries)
    const u32 per = (len + FIN_THREADS - 1) / FIN_THREADS;
    const u32 b0 = min(len, tid * per), b1 = min(len, b0 + per);
    u64 kk[FIN_ITEMS];
    u32 rr[FIN_ITEMS];
    u32 lt = 0, eq = 0;
#pragma unroll
    for (int j = 0; j < FIN_ITEMS; ++j) {
      const u32 o = b0 + (u32)j;
      if (o < b1) {
        kk[j] = sm.skeys[s + o];
        rr[j] = sm.srids[s + o];
        lt += kk[j] < piv;
        eq += kk[j] == piv;
      }
    }
    u32 tot;
    const u32 ex = block_excl_sum<FIN_WAVES>(lt | (eq << 16), sm.scan, &tot);  // ends with a barrier
    const u32 LT = tot & 0xFFFFu, EQ = tot >> 16;
    u32 plt = s + (ex & 0xFFFFu), peq = s + LT + (ex >> 16);
    u32 pgt = s + LT + EQ + (b0 - (ex & 0xFFFFu) - (ex >> 16));
#pragma unroll
    for (int j = 0; j < FIN_ITEMS; ++j) {
      const u32 o = b0 + (u32)j;
      if (o < b1) {
        const u32 d = kk[j] < piv ? plt++ : (kk[j] == piv ? peq++ : pgt++);
        sm.skeys[d] = kk[j];
        sm.srids[d] = rr[j];
      }
    }
    __syncthreads();
    // the parts below and above the pivot
    const u32 part_lo[2] = {s, s + LT + EQ};
    const u32 part_hi[2] = {s + LT, e};
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const u32 pl = part_lo[q], ph = part_hi[q];
      if (ph - pl <= 1) continue;
      if (ph - pl <= SHORT_RUN) {
        rank_short(sm, pl, ph);
      } else if (tid == 0) {
        const u32 idx = sm.n_long;
        if (idx < LONG_RUNS) {
          sm.long_lo[idx] = pl;
          sm.long_hi[idx] = ph;
          sm.n_long = idx + 1;
        } else {
          sm.flag = 1;
        }
      }
    }
    __syncthreads();
  }
}

enum ChunkResult : u32 { CH_EQUAL = 0, CH_INORDER = 1, CH_MOVED = 2 };

// Stable on-chip sort of the chunk [0, m) in sm using the model once more:
// entries are ranked by their refined bucket id (8 more bits of F, given in
// sm.srel, taken relative to the chunk's first bucket) in one or two byte
// passes, which leaves runs of entries sharing a refined id -- a handful each
// when the model fits -- that are sorted by key.  The m <= FIN_THREADS*IT
// entries are spread over IT items per thread, so that every wave has work
// whatever the chunk's size.  A long run of distinct keys the three-way
// splits cannot settle sends the chunk to the byte-wise LSD sort.  Returns
// CH_EQUAL when all keys are equal and CH_INORDER when they already ascend
// (nothing moved in either case).
template <int IT>
__device__ u32 lds_sort_model(FinishSmem& sm, const SegModel& m, u32 mcount) {
  const u32 tid = threadIdx.x;
  const u32 w = tid >> 6;
  u64 vor = 0, vand = ~0ull;
  u32 rmax = 0;  // largest refined id relative to the chunk's first bucket
  bool inv = false;  // some entry's key is below its predecessor's
  // sm.srel holds each entry's refined bucket id (the first rank pass makes
  // it relative to the chunk's first bucket)
  const u32 base = (sm.srel[0] >> REFINE_BITS) << REFINE_BITS;
  for (u32 i = tid; i < mcount; i += FIN_THREADS) {
    const u64 k = sm.skeys[i];
    vor |= k;
    vand &= k;
    const u32 r = sm.srel[i] - base;
    rmax = r > rmax ? r : rmax;
    inv = inv || (i > 0 && k < sm.skeys[i - 1]);
  }
  // one block reduction of all four (a single barrier)
  vor = wave_reduce(vor, (u64)0, [](u64 x, u64 y) { return x | y; });
  vand = wave_reduce(vand, ~(u64)0, [](u64 x, u64 y) { return x & y; });
  rmax = wave_reduce(rmax, 0u, [](u32 x, u32 y) { return x > y ? x : y; });
  const bool winv = ballot(inv) != 0;
  if (__lane_id() == 0) {
    sm.red64[w] = vor;
    sm.red64[FIN_WAVES + w] = vand;
    sm.red[w] = rmax;
    sm.red_inv[w] = winv ? 1u : 0u;
  }
  __syncthreads();
  inv = false;
#pragma unroll
  for (int q = 0; q < FIN_WAVES; ++q) {
    vor |= sm.red64[q];
    vand &= sm.red64[FIN_WAVES + q];
    rmax = sm.red[q] > rmax ? sm.red[q] : rmax;
    inv = inv || sm.red_inv[q] != 0;
  }
  if (vor == vand) return CH_EQUAL;
  if (!inv) return CH_INORDER;
  if (!m.valid || rmax >= (1u << 16)) {
    lds_sort(sm, mcount);
    return CH_MOVED;
  }
  u32 valid = 0;
#pragma unroll
  for (int j = 0; j < IT; ++j)
    if (part_offset<FIN_WAVES, IT>(j) < mcount) valid |= 1u << j;
#pragma unroll 1
  for (u32 p = 0; p < 2; ++p) {
    if (p == 1 && rmax < 256u) break;
    u64 kk[IT];
    u32 rr[IT], re[IT], d[IT], rank[IT], tc;
#pragma unroll
    for (int j = 0; j < IT; ++j) {
      const u32 o = part_offset<FIN_WAVES, IT>(j);
      const bool v = (valid >> j) & 1;
      kk[j] = v ? sm.skeys[o] : 0ull;
      rr[j] = v ? sm.srids[o] : 0u;
      re[j] = v ? sm.srel[o] - (p == 0 ? base : 0u) : 0u;
      d[j] = (re[j] >> (8 * p)) & 255u;
    }
    // items read before rank_tile's first barrier, overwritten after its last;
    // a pass's digits are below 2^nbits (the second pass's: the chunk's
    // bucket offset, a few bits)
    const u32 top = p == 0 ? (rmax < 256u ? rmax : 255u) : (rmax >> 8);
    const u32 nbits = top ? 32u - __clz(top) : 1u;
    rank_tile(sm.whist, sm.lstart, sm.scan, d, valid, rank, &tc, nbits);
#pragma unroll
    for (int j = 0; j < IT; ++j)
      if ((valid >> j) & 1) {
        const u32 pos = sm.lstart[d[j]] + sm.whist[w][d[j]] + rank[j];
        sm.skeys[pos] = kk[j];
        sm.srids[pos] = rr[j];
        sm.srel[pos] = re[j];
      }
    __syncthreads();
  }
  // Runs of equal refined id: run starts, run ends and adjacent inversions
  // are found in parallel; each entry of a short run with an inversion counts
  // the run's entries that must precede it; a long run is left alone when it
  // has no inversion (typically one repeated key) and is otherwise split
  // three ways around a sampled pivot.
  if (tid == 0) {
    sm.flag = 0;
    sm.n_long = 0;
  }
  u32 stm = 0, lastm = 0, invm = 0, rs[IT];
  u32 carry = 0;
  const u32 lane = __lane_id();
#pragma unroll
  for (int j = 0; j < IT; ++j) {
    const u32 i = part_offset<FIN_WAVES, IT>(j);
    bool st = false, la = false, inv = false;
    if (i < mcount) {
      const u32 r = sm.srel[i];
      st = i == 0 || sm.srel[i - 1] != r;
      la = i + 1 == mcount || sm.srel[i + 1] != r;
      inv = !st && sm.skeys[i] < sm.skeys[i - 1];
    }
    stm |= (u32)st << j;
    lastm |= (u32)la << j;
    invm |= (u32)inv << j;
    // run start of position i: max start position <= i (wave scan + carry)
    u32 v = wave_incl_scan(st ? i : 0u, 0u, [](u32 x, u32 y) { return x > y ? x : y; });
    v = carry > v ? carry : v;
    rs[j] = v;
    carry = lane63(v);
  }
  // earlier waves' last run start
  sm.red[w] = carry;
  __syncthreads();
  u32 before = 0;
  for (u32 q = 0; q < w; ++q) before = sm.red[q] > before ? sm.red[q] : before;
#pragma unroll
  for (int j = 0; j < IT; ++j) rs[j] = rs[j] > before ? rs[j] : before;
  __syncthreads();
  // the last entry of each run stores the run's end at the run's start; an
  // inversion inside a run marks the run (bit 31) as needing the sort
#pragma unroll
  for (int j = 0; j < IT; ++j)
    if ((lastm >> j) & 1) sm.srel[rs[j]] = part_offset<FIN_WAVES, IT>(j) + 1;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < IT; ++j)
    if ((invm >> j) & 1) atomicOr(&sm.srel[rs[j]], 0x80000000u);
  __syncthreads();
  // Each entry of a short run counts the run's entries that must precede it
  // (smaller key, or equal key earlier): its position within the run.
  u64 nk[IT];
  u32 nr[IT], np[IT];
  u32 movem = 0;
#pragma unroll
  for (int j = 0; j < IT; ++j) {
    const u32 i = part_offset<FIN_WAVES, IT>(j);
    np[j] = i;
    if (i >= mcount) continue;
    const u32 s0 = rs[j], re = sm.srel[s0], e = re & 0x7FFFFFFFu;
    if (!(re >> 31)) continue;  // run already in order
    if (e - s0 > SHORT_RUN) {
      if (i == s0) {  // the run's start registers it for the three-way splits
        const u32 idx = atomicAdd(&sm.n_long, 1u);
        if (idx < LONG_RUNS) {
          sm.long_lo[idx] = s0;
          sm.long_hi[idx] = e;
        } else {
          sm.flag = 1;
        }
      }
      continue;
    }
    const u64 k = sm.skeys[i];
    u32 rank = 0;
    for (u32 q = s0; q < e; ++q) {
      const u64 kq = sm.skeys[q];
      rank += (kq < k) || (kq == k && q < i);
    }
    np[j] = s0 + rank;
    nk[j] = k;
    nr[j] = sm.srids[i];
    movem |= (u32)(np[j] != i) << j;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < IT; ++j)
    if ((movem >> j) & 1) {
      sm.skeys[np[j]] = nk[j];
      sm.srids[np[j]] = nr[j];
    }
  __syncthreads();
  if (!sm.flag) split_long_runs(sm);
  if (sm.flag) lds_sort(sm, mcount);
  return CH_MOVED;
}

// Finishing pass over the 2048-entry stretches [pos0, pos0+FH) of every
// segment.  A stretch owns the buckets whose first entry lies in it: the
// chunk [start, end) from its first bucket start to the first bucket start at
// or after pos0+FH (or the segment end).  Chunks of at most FCAP entries are
// sorted on chip; larger ones are listed for the pivot rounds.
//
// Step 1 (k_fin_active, one thread per stretch): bucket ids never decrease
// along a segment, so a stretch other than a segment's first holds a bucket
// start exactly when the entry before it and its last entry lie in different
// buckets; its first bucket start is then found by binary search.  edge[t]
// is that start's offset in stretch t (0 for a segment's first stretch),
// NONE when the stretch holds none.  The stretches that hold one are listed
// (about half of them on skewed keys); the rest need no work.  A listed
// stretch is (segment << 32 | index in the segment), so that its workgroup
// needs no lookup before the segment's data.
__global__ void __launch_bounds__(BLOCK) k_fin_active(const u64* __restrict__ keys, SegList sl,
                                                      const u32* __restrict__ ftile_start,
                                                      const u32* __restrict__ ftile_seg,
                                                      const SegModel* __restrict__ segm,
                                                      u32 max_ftiles, u32* __restrict__ edge,
                                                      u64* __restrict__ active,
                                                      u32* __restrict__ n_active) {
  const u32 n_seg = sl.n();
  const u32 total = min(ftile_start[n_seg], max_ftiles);
  for (u32 t0 = blockIdx.x * BLOCK; t0 < total; t0 += gridDim.x * BLOCK) {
    const u32 tile = t0 + threadIdx.x;
    u32 e = NONE;
    u64 item = 0;
    if (tile < total) {
      const u32 seg = ftile_seg[tile];
      const u32 k = tile - ftile_start[seg];
      item = ((u64)seg << 32) | k;
      const u64 a = sl.lo[seg], b = sl.hi[seg];
      const u64 pos0 = a + (u64)k * FH;
      if (pos0 < b) {
        if (k == 0) {
          e = 0;
        } else {
          const SegModel m = segm[seg];
          const u32 span = (u32)min<u64>(FH, b - pos0);
          const global_float* gk = (const global_float*)m.knots;
          const u32 b0 = model_bucket(m, gk, keys[pos0 - 1]);
          if (model_bucket(m, gk, keys[pos0 - 1 + span]) != b0) {
            // first offset o in [1, span] whose entry pos0 - 1 + o leaves bucket b0
            u32 lo = 1, hi = span;
            while (lo < hi) {
              const u32 mid = (lo + hi) >> 1;
              if (model_bucket(m, gk, keys[pos0 - 1 + mid]) != b0) hi = mid; else lo = mid + 1;
            }
            e = lo - 1;
          }
        }
      }
      edge[tile] = e;
    }
    const bool act = e != NONE;
    const u64 bal = ballot(act);
    u32 wbase = 0;
    if (__lane_id() == 0 && bal) wbase = atomicAdd(n_active, (u32)__popcll(bal));
    wbase = __shfl(wbase, 0, 64);
    if (act) active[wbase + (u32)__popcll(bal & lanemask_lt())] = item;
  }
}

// Step 2: one listed stretch's chunk.  Its start is the stretch's first
// bucket start; its end, the first bucket start of a later stretch of the
// segment (edge[], read FIN_THREADS stretches at a time) or the segment end.
// The workgroup reads the chunk's keys (and row ids); every return is
// uniform over the workgroup.
//
// VALS: the chunk also carries a value column.  The on-chip sort then
// orders local indices instead of row ids; the chunk's row ids and values
// are loaded into registers while the sorted keys are written, and go
// through the free LDS areas into the new order.
// Permutes the row ids and values of [start, start + m) in place by the local
// indices in sm.srids (sm.srids[i] = old position of the entry now at i).
// The caller has written the sorted keys; begins with a barrier.
__device__ __forceinline__ void permute_rids_vals(FinishSmem& sm, u32* __restrict__ rids,
                                                  u64* __restrict__ vals, u64 start, u32 m) {
  __syncthreads();  // every thread has read the sorted keys from sm.skeys
  for (u32 i = threadIdx.x; i < m; i += FIN_THREADS) {
    sm.skeys[i] = vals[start + i];
    sm.srel[i] = rids[start + i];
  }
  __syncthreads();
  for (u32 i = threadIdx.x; i < m; i += FIN_THREADS) {
    const u32 o = sm.srids[i];
    vals[start + i] = sm.skeys[o];
    rids[start + i] = sm.srel[o];
  }
}

template <bool VALS>
__device__ __forceinline__ void finish_stretch(
    FinishSmem& sm, u64* __restrict__ keys, u32* __restrict__ rids, u64* __restrict__ vals,
    const SegList& sl, const u32* __restrict__ ftile_start, const u32* __restrict__ edge,
    const SegModel* __restrict__ segm, u64* __restrict__ fb_lo, u64* __restrict__ fb_hi,
    u32* __restrict__ fb_seg, u32* __restrict__ fb_count, u32 max_fb, kpa_sort_stats* stats,
    u64 item) {
  const u32 tid = threadIdx.x;
  const u32 seg = (u32)(item >> 32);
  const u32 k = (u32)item;
  const u64 a = sl.lo[seg], b = sl.hi[seg];
  const u64 pos0 = a + (u64)k * FH;
  if (pos0 >= b) return;
  const u32 f0 = ftile_start[seg];
  const u32 nst = (u32)((b - a + FH - 1) / FH);  // stretches holding entries
  const u64 start = pos0 + edge[f0 + k];
  u64 end = b;
  for (u32 k2 = k + 1; k2 < nst; k2 += FIN_THREADS) {
    const u32 kk = k2 + tid;
    const bool found = kk < nst && edge[f0 + kk] != NONE;
    const u32 first = block_min_u32<FIN_WAVES>(found ? tid : NONE, sm.red);
    if (first != NONE) {
      end = a + (u64)(k2 + first) * FH + edge[f0 + k2 + first];
      break;
    }
  }
  if (end - start > FCAP) {  // oversize: listed for the pivot rounds
    if (tid == 0) {
      const u32 idx = atomicAdd(fb_count, 1u);
      if (idx < max_fb) {
        fb_lo[idx] = start;
        fb_hi[idx] = end;
        fb_seg[idx] = seg;
      }
    }
    return;
  }
  const u32 mcount = (u32)(end - start);  // <= FCAP
  const SegModel m = segm[seg];
  {
    constexpr int IT = (int)(FCAP / FIN_THREADS);
    u64 kv[IT];  // in flight while the knots are copied to LDS
    u32 rv[IT];
#pragma unroll
    for (int j = 0; j < IT; ++j) {
      const u32 i = tid + j * FIN_THREADS;
      kv[j] = i < mcount ? keys[start + i] : 0ull;
      rv[j] = VALS ? i : (i < mcount ? rids[start + i] : 0u);
    }
    const lds_float* kn = bind_knots(m, sm.knots);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < IT; ++j) {
      const u32 i = tid + j * FIN_THREADS;
      if (i < mcount) {
        sm.skeys[i] = kv[j];
        sm.srids[i] = rv[j];
        sm.srel[i] = m.valid ? model_fine(m, kn, kv[j]) : 0u;
      }
    }
  }
  __syncthreads();  // the sort reads other threads' entries before its first barrier
  u32 res;
  if (mcount <= 2048)
    res = lds_sort_model<4>(sm, m, mcount);
  else if (mcount <= 3072)
    res = lds_sort_model<6>(sm, m, mcount);
  else
    res = lds_sort_model<8>(sm, m, mcount);
  if (tid == 0) stat_add(stats, res == CH_EQUAL ? ST_EQUAL : ST_ONCHIP, mcount);
  if (res != CH_MOVED) return;
  if (VALS) {
    // The chunk's row ids and values are loaded into registers (entry
    // tid + j*FIN_THREADS in slot j) while the sorted keys are written, then
    // go through the free LDS areas into the new order.
    constexpr int PF = (int)(FCAP / FIN_THREADS);
    static_assert(FCAP % FIN_THREADS == 0, "a chunk spreads evenly over the threads");
    u64 pv[PF];
    u32 pr[PF];
#pragma unroll
    for (int j = 0; j < PF; ++j) {
      const u32 i = tid + j * FIN_THREADS;
      pv[j] = i < mcount ? vals[start + i] : 0ull;
      pr[j] = i < mcount ? rids[start + i] : 0u;
    }
    for (u32 i = tid; i < mcount; i += FIN_THREADS) keys[start + i] = sm.skeys[i];
    __syncthreads();  // every thread has read the sorted keys
#pragma unroll
    for (int j = 0; j < PF; ++j) {
      const u32 i = tid + j * FIN_THREADS;
      if (i < mcount) {
        sm.skeys[i] = pv[j];
        sm.srel[i] = pr[j];
      }
    }
    __syncthreads();
    for (u32 i = tid; i < mcount; i += FIN_THREADS) {
      const u32 o = sm.srids[i];  // old position of the entry now at i
      vals[start + i] = sm.skeys[o];
      rids[start + i] = sm.srel[o];
    }
    return;
  }
  for (u32 i = tid; i < mcount; i += FIN_THREADS) {
    keys[start + i] = sm.skeys[i];
    rids[start + i] = sm.srids[i];
  }
}

// One workgroup per listed stretch (the grid covers every stretch; the
// workgroups past the list's end return at once).  A persistent loop over the
// list needs more registers than the body alone and measured slower.
template <bool VALS>
__global__ void __launch_bounds__(FIN_THREADS, 4) k_learned_finish(
    u64* __restrict__ keys, u32* __restrict__ rids, u64* __restrict__ vals, SegList sl,
    const u32* __restrict__ ftile_start, const u32* __restrict__ edge,
    const SegModel* __restrict__ segm, const u64* __restrict__ active,
    const u32* __restrict__ n_active, u64* __restrict__ fb_lo, u64* __restrict__ fb_hi,
    u32* __restrict__ fb_seg, u32* __restrict__ fb_count, u32 max_fb, kpa_sort_stats* stats) {
  __shared__ FinishSmem sm;
  if (blockIdx.x >= *n_active) return;
  finish_stretch<VALS>(sm, keys, rids, vals, sl, ftile_start, edge, segm, fb_lo, fb_hi, fb_seg,
                       fb_count, max_fb, stats, active[blockIdx.x]);
}

// Sorts listed ranges of at most FCAP entries in place, one workgroup each.
// A range is a part of an oversize chunk, in bucket order; above FIN_THREADS
// entries it is sorted as a finishing chunk is, by its segment's refined
// bucket ids and then within runs of equal id.
template <bool VALS>
__global__ void __launch_bounds__(FIN_THREADS, 4) k_lds_sort_ranges(u64* __restrict__ keys,
                                                           u32* __restrict__ rids,
                                                           u64* __restrict__ vals,
                                                           const u64* __restrict__ lo,
                                                           const u64* __restrict__ hi,
                                                           const u32* __restrict__ seg,
                                                           const SegModel* __restrict__ segm,
                                                           const u32* __restrict__ count,
                                                           u32 max_count) {
  __shared__ FinishSmem sm;
  const u32 n = min(*count, max_count);
  for (u32 r = blockIdx.x; r < n; r += gridDim.x) {
    const u64 a = lo[r];
    const u32 m = (u32)(hi[r] - a);
    __syncthreads();
    bool moved;
    if (m <= FIN_THREADS) {
      for (u32 i = threadIdx.x; i < m; i += FIN_THREADS) {
        sm.skeys[i] = keys[a + i];
        sm.srids[i] = VALS ? i : rids[a + i];
      }
      moved = rank_sort_small(sm, m);
    } else {
      const SegModel md = segm[seg[r]];
      const lds_float* kn = md.valid ? bind_knots(md, sm.knots) : nullptr;
      __syncthreads();
      for (u32 i = threadIdx.x; i < m; i += FIN_THREADS) {
        const u64 k = keys[a + i];
        sm.skeys[i] = k;
        sm.srids[i] = VALS ? i : rids[a + i];
        sm.srel[i] = md.valid ? model_fine(md, kn, k) : 0u;
      }
      __syncthreads();  // the sort reads other threads' entries before its first barrier
      u32 res;
      if (m <= 2048)
        res = lds_sort_model<4>(sm, md, m);
      else if (m <= 3072)
        res = lds_sort_model<6>(sm, md, m);
      else
        res = lds_sort_model<8>(sm, md, m);
      moved = res == CH_MOVED;
    }
    if (moved) {
      if (VALS) {
        for (u32 i = threadIdx.x; i < m; i += FIN_THREADS) keys[a + i] = sm.skeys[i];
        permute_rids_vals(sm, rids, vals, a, m);
      } else {
        for (u32 i = threadIdx.x; i < m; i += FIN_THREADS) {
          keys[a + i] = sm.skeys[i];
          rids[a + i] = sm.srids[i];
        }
      }
    }
  }
}

// ----------------------------------------------------------- pivot rounds --

// Pivot of each listed chunk: the most frequent of 256 evenly spaced keys
// (ties: the smaller key).  Also clears the chunk's counters.
__global__ void __launch_bounds__(BLOCK) k_fb_pivot(const u64* __restrict__ keys, SegList sl,
                                                    u64* __restrict__ pivot,
                                                    u64* __restrict__ cnt3) {
  __shared__ u64 samp[BLOCK];
  __shared__ u64 bk[WAVES];
  __shared__ u32 bc[WAVES];
  const u32 n = sl.n();
  for (u32 c = blockIdx.x; c < n; c += gridDim.x) {
    const u64 a = sl.lo[c], m = sl.hi[c] - a;
    __syncthreads();
    samp[threadIdx.x] = keys[a + (m - 1) * threadIdx.x / (BLOCK - 1)];
    __syncthreads();
    const u64 mine = samp[threadIdx.x];
    u32 cnt = 0;
    for (int i = 0; i < BLOCK; ++i) cnt += samp[i] == mine;
    // block argmax over (count desc, key asc)
    u64 key = mine;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const u32 oc = __shfl_xor(cnt, o, 64);
      const u64 okey = __shfl_xor(key, o, 64);
      if (oc > cnt || (oc == cnt && okey < key)) {
        cnt = oc;
        key = okey;
      }
    }
    if (__lane_id() == 0) {
      bc[threadIdx.x >> 6] = cnt;
      bk[threadIdx.x >> 6] = key;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      u32 best = bc[0];
      u64 bkey = bk[0];
      for (int i = 1; i < WAVES; ++i)
        if (bc[i] > best || (bc[i] == best && bk[i] < bkey)) {
          best = bc[i];
          bkey = bk[i];
        }
      pivot[c] = bkey;
      cnt3[3 * c] = cnt3[3 * c + 1] = cnt3[3 * c + 2] = 0;
    }
  }
}

// Entries below / equal to the pivot, per tile of the chunk list and per
// chunk (comparisons and wave sums; one atomic pair per tile).  Each thread
// also stores which of its entries (tile_offset layout) equal the pivot, so
// that the move reads no key of the equal part and the copy back writes the
// pivot only where another key stood.
__global__ void __launch_bounds__(BLOCK) k_fb_count(const u64* __restrict__ keys, SegList sl,
                                                    const u32* __restrict__ tile_start,
                                                    const u32* __restrict__ tile_seg,
                                                    const u64* __restrict__ pivot,
                                                    u64* __restrict__ cnt3,
                                                    u32* __restrict__ t_lt,
                                                    u32* __restrict__ t_eq,
                                                    uint16_t* __restrict__ t_eqbits) {
  static_assert(ITEMS <= 16, "one 16-bit word of flags per thread and tile");
  __shared__ u64 red[2 * WAVES];
  const u32 n_seg = sl.n();
  const u32 total = tile_start[n_seg];
  for (u32 tile = blockIdx.x; tile < total; tile += gridDim.x) {
    u32 seg, t_in, cnt;
    u64 a, b, base;
    seg_tile_range(sl, tile_start, n_seg, tile, seg, t_in, a, b, base, cnt, tile_seg);
    const u64 h = pivot[seg];
    u64 lt = 0, eq = 0;
    u64 kv[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const u32 o = tile_offset(j);
      kv[j] = o < cnt ? keys[base + o] : 0ull;
    }
    u32 eqbits = 0;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      if (tile_offset(j) < cnt) {
        lt += kv[j] < h;
        eq += kv[j] == h;
        eqbits |= (u32)(kv[j] == h) << j;
      }
    }
    t_eqbits[(u64)tile * BLOCK + threadIdx.x] = (uint16_t)eqbits;
    lt = wave_sum(lt);
    eq = wave_sum(eq);
    __syncthreads();
    if (__lane_id() == 0) {
      red[threadIdx.x >> 6] = lt;
      red[WAVES + (threadIdx.x >> 6)] = eq;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      u64 l = 0, e = 0;
      for (int i = 0; i < WAVES; ++i) {
        l += red[i];
        e += red[WAVES + i];
      }
      t_lt[tile] = (u32)l;
      t_eq[tile] = (u32)e;
      if (cnt) {
        atomicAdd(reinterpret_cast<unsigned long long*>(cnt3 + 3 * seg), (unsigned long long)l);
        atomicAdd(reinterpret_cast<unsigned long long*>(cnt3 + 3 * seg + 1), (unsigned long long)e);
      }
    }
  }
}

// One thread per chunk: whether the chunk
// needs the scatter at all (not when it holds only the pivot key), and the
// parts still to sort: on chip when small, else in the next round.
__global__ void __launch_bounds__(BLOCK) k_fb_plan(SegList sl, const u32* __restrict__ c_seg,
                                                   const u64* __restrict__ cnt3,
                                                   u32* __restrict__ p_mask,
                                                   u64* __restrict__ sm_lo, u64* __restrict__ sm_hi,
                                                   u32* __restrict__ sm_seg,
                                                   u32* __restrict__ sm_count, u32 sm_max,
                                                   u64* __restrict__ nx_lo, u64* __restrict__ nx_hi,
                                                   u32* __restrict__ nx_seg,
                                                   u32* __restrict__ nx_count, u32 nx_max,
                                                   kpa_sort_stats* stats) {
  const u32 n = sl.n();
  for (u32 c = blockIdx.x * BLOCK + threadIdx.x; c < n; c += gridDim.x * BLOCK) {
    const u64 a = sl.lo[c], m = sl.hi[c] - a;
    const u64 lt = cnt3[3 * c], eq = cnt3[3 * c + 1];
    const u64 gt = m - lt - eq;
    const bool pure = eq == m;
    p_mask[c] = pure ? 0u : 1u;
    if (stats) {
      stat_add(stats, ST_EQUAL, eq);
      stat_add(stats, ST_FB_ENTRIES, m - eq);
      if (!pure) stat_add(stats, ST_FB_BUCKETS, 1);
    }
    const u64 parts_lo[2] = {a, a + lt + eq};
    const u64 parts_n[2] = {lt, gt};
    for (int p = 0; p < 2; ++p) {
      if (parts_n[p] < 2) continue;
      if (parts_n[p] <= FCAP) {
        const u32 i = atomicAdd(sm_count, 1u);
        if (i < sm_max) {
          sm_lo[i] = parts_lo[p];
          sm_hi[i] = parts_lo[p] + parts_n[p];
          sm_seg[i] = c_seg[c];
        }
      } else {
        const u32 i = atomicAdd(nx_count, 1u);
        if (i < nx_max) {
          nx_lo[i] = parts_lo[p];
          nx_hi[i] = parts_lo[p] + parts_n[p];
          nx_seg[i] = c_seg[c];
        }
      }
    }
  }
}

// Per chunk to split (one workgroup each): the counts of entries below and
// equal to the pivot in the chunk's earlier tiles (exclusive prefix over its
// tiles, in place).
__global__ void __launch_bounds__(1024) k_fb_tscan(SegList sl, const u32* __restrict__ tile_start,
                                                   const u32* __restrict__ p_mask,
                                                   u32* __restrict__ t_lt, u32* __restrict__ t_eq) {
  __shared__ u32 sm[17];
  const u32 n = sl.n();
  for (u32 c = blockIdx.x; c < n; c += gridDim.x) {
    if (!p_mask[c]) continue;
    const u32 t0 = tile_start[c], t1 = tile_start[c + 1];
    u32 cl = 0, ce = 0;
    for (u32 b = t0; b < t1; b += 1024) {
      const u32 t = b + threadIdx.x;
      const u32 vl = t < t1 ? t_lt[t] : 0u, ve = t < t1 ? t_eq[t] : 0u;
      u32 tl, te;
      const u32 xl = block_excl_sum<16>(vl, sm, &tl);
      const u32 xe = block_excl_sum<16>(ve, sm, &te);
      if (t < t1) {
        t_lt[t] = cl + xl;
        t_eq[t] = ce + xe;
      }
      cl += tl;
      ce += te;
    }
  }
}

// Stable three-way split of a chunk [a, b) around its pivot h, into the
// temporary buffers at the final positions: entries below h go to
// [a, a+LT), entries above to [a+LT+EQ, b) (keys and row ids), entries equal
// to h only send their row ids to [a+LT, a+LT+EQ) (their keys are all h).
// An entry's place in its class: the class's count in earlier tiles (tscan)
// plus its stable rank in the tile (ballot ranks per wave, offsets across
// waves).
__global__ void __launch_bounds__(BLOCK) k_fb_move(const u64* __restrict__ keys,
                                                   const u32* __restrict__ rids, SegList sl,
                                                   const u32* __restrict__ tile_start,
                                                   const u32* __restrict__ tile_seg,
                                                   const u64* __restrict__ pivot,
                                                   const u64* __restrict__ cnt3,
                                                   const u32* __restrict__ p_mask,
                                                   const u32* __restrict__ t_lt,
                                                   const u32* __restrict__ t_eq,
                                                   const uint16_t* __restrict__ t_eqbits,
                                                   u64* __restrict__ keys_tmp,
                                                   u32* __restrict__ rids_tmp,
                                                   const u64* __restrict__ vals,
                                                   u64* __restrict__ vals_tmp) {
  __shared__ u32 whist[WAVES][RADIX];
  const u32 n_seg = sl.n();
  const u32 total = tile_start[n_seg];
  const u32 w = threadIdx.x >> 6;
  for (u32 tile = blockIdx.x; tile < total; tile += gridDim.x) {
    u32 seg, t_in, cnt;
    u64 a, b, base;
    seg_tile_range(sl, tile_start, n_seg, tile, seg, t_in, a, b, base, cnt, tile_seg);
    if (!p_mask[seg]) continue;
    const u64 h = pivot[seg];
    u64 kk[ITEMS];
    u32 rr[ITEMS], d[ITEMS], rank[ITEMS];
    u32 valid = 0;
    const u32 eqbits = t_eqbits[(u64)tile * BLOCK + threadIdx.x];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const u32 o = tile_offset(j);
      kk[j] = h;
      rr[j] = 0;
      if (o < cnt) {
        if (!((eqbits >> j) & 1)) kk[j] = keys[base + o];  // the equal part's keys are the pivot
        rr[j] = rids[base + o];
        valid |= 1u << j;
      }
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) d[j] = ((eqbits >> j) & 1) ? 1u : (kk[j] < h ? 0u : 2u);
    __syncthreads();  // the previous tile's whist reads are done
    rank_count<WAVES, ITEMS>(whist, d, valid, rank, 2);  // classes 0..2: two digit bits
    __syncthreads();  // rank_count turns the counts into cross-wave offsets after its barrier
    const u32 lt0 = t_lt[tile], eq0 = t_eq[tile];
    const u64 LT = cnt3[3 * seg], EQ = cnt3[3 * seg + 1];
    const u64 start[3] = {a + lt0, a + LT + eq0, a + LT + EQ + ((u64)t_in * TILE - lt0 - eq0)};
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      if ((valid >> j) & 1) {
        const u64 dst = start[d[j]] + whist[w][d[j]] + rank[j];
        rids_tmp[dst] = rr[j];
        if (d[j] != 1) keys_tmp[dst] = kk[j];
        if (vals) vals_tmp[dst] = vals[base + tile_offset(j)];
      }
    }
  }
}

// The split chunks back into place: row ids from the temporary buffer; keys
// from it too, except in the equal part, which is the pivot: written only
// where the chunk held another key before the split (the flags of k_fb_count
// describe the entries at the same positions, in the same thread layout).
__global__ void __launch_bounds__(BLOCK) k_fb_back(u64* __restrict__ keys, u32* __restrict__ rids,
                                                   SegList sl, const u32* __restrict__ tile_start,
                                                   const u32* __restrict__ tile_seg,
                                                   const u64* __restrict__ pivot,
                                                   const u64* __restrict__ cnt3,
                                                   const u32* __restrict__ p_mask,
                                                   const uint16_t* __restrict__ t_eqbits,
                                                   const u64* __restrict__ keys_tmp,
                                                   const u32* __restrict__ rids_tmp,
                                                   u64* __restrict__ vals,
                                                   const u64* __restrict__ vals_tmp) {
  const u32 n_seg = sl.n();
  const u32 total = tile_start[n_seg];
  for (u32 tile = blockIdx.x; tile < total; tile += gridDim.x) {
    u32 seg, t_in, cnt;
    u64 a, b, base;
    seg_tile_range(sl, tile_start, n_seg, tile, seg, t_in, a, b, base, cnt, tile_seg);
    if (!p_mask[seg]) continue;
    const u64 h = pivot[seg];
    const u64 e0 = a + cnt3[3 * seg], e1 = e0 + cnt3[3 * seg + 1];
    const u32 eqbits = t_eqbits[(u64)tile * BLOCK + threadIdx.x];
    u64 kv[ITEMS];
    u32 rv[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const u64 p = base + tile_offset(j);
      const bool in = tile_offset(j) < cnt;
      rv[j] = in ? rids_tmp[p] : 0u;
      kv[j] = (in && (p < e0 || p >= e1)) ? keys_tmp[p] : h;
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const u64 p = base + tile_offset(j);
      if (tile_offset(j) < cnt) {
        rids[p] = rv[j];
        if (vals) vals[p] = vals_tmp[p];
        // in the equal part the pivot is already there where the chunk held it
        if (p < e0 || p >= e1 || !((eqbits >> j) & 1)) keys[p] = kv[j];
      }
    }
  }
}

kpa_status learned_sort_plan(u64 n_cap, u32 n_seg, Carver& c, LearnedWs* w, bool vals) {
  w->n_cap = n_cap;
  w->max_tiles = max_tiles(n_cap, n_seg, TILE);
  w->max_ftiles = max_tiles(n_cap, n_seg, FH);
  // an oversize chunk holds more than FCAP entries
  w->max_fb = (u32)(n_cap / FCAP + n_seg + 1);
  w->keys_tmp = c.take<u64>(n_cap);
  w->rids_tmp = c.take<u32>(n_cap);
  w->vals_tmp = vals ? c.take<u64>(n_cap) : nullptr;
  w->segm = c.take<SegModel>(n_seg);
  w->cur_min = c.take<u64>(n_seg);
  w->cur_max = c.take<u64>(n_seg);
  w->ltile_start = c.take<u32>((u64)n_seg + 1);
  w->ftile_start = c.take<u32>((u64)n_seg + 1);
  w->ltile_seg = c.take<u32>(w->max_tiles);
  w->ftile_seg = c.take<u32>(w->max_ftiles);
  w->factive = c.take<u64>(w->max_ftiles);
  w->fedge = c.take<u32>(w->max_ftiles);
  w->fn_active = c.take<u32>(1);
  w->hist = c.take<u32>((u64)n_seg * 2 * RADIX);
  w->seg_mask = c.take<u32>(n_seg);
  w->status0 = c.take<u32>(w->max_tiles * RADIX);
  w->status1 = c.take<u32>(w->max_tiles * RADIX);
  w->counters = c.take<u32>(16);
  order_plan(c, w->max_tiles, n_seg, &w->order);
  w->fb_lo = c.take<u64>(w->max_fb);
  w->fb_hi = c.take<u64>(w->max_fb);
  w->fb_seg = c.take<u32>(w->max_fb);
  w->fb_min = c.take<u64>(1);
  w->fb_max = c.take<u64>(1);
  w->fb_count = c.take<u32>(1);
  w->fb_tile_start = c.take<u32>((u64)w->max_fb + 1);
  w->fb_tile_seg = c.take<u32>(max_tiles(n_cap, w->max_fb, TILE));
  for (int r = 0; r < 2; ++r) {
    w->rl_lo[r] = c.take<u64>(w->max_fb);
    w->rl_hi[r] = c.take<u64>(w->max_fb);
    w->rl_seg[r] = c.take<u32>(w->max_fb);
  }
  w->rl_count = c.take<u32>(4);
  w->sm_lo = c.take<u64>(6ull * w->max_fb);
  w->sm_hi = c.take<u64>(6ull * w->max_fb);
  w->sm_seg = c.take<u32>(6ull * w->max_fb);
  w->pivot = c.take<u64>(w->max_fb);
  w->cnt3 = c.take<u64>(3ull * w->max_fb);
  w->p_mask = c.take<u32>(w->max_fb);
  w->t_lt = c.take<u32>(max_tiles(n_cap, w->max_fb, TILE));
  w->t_eq = c.take<u32>(max_tiles(n_cap, w->max_fb, TILE));
  w->t_eqbits = c.take<uint16_t>(max_tiles(n_cap, w->max_fb, TILE) * BLOCK);
  // The radix path for what the pivot rounds leave: its own ping-pong buffer
  // and per-chunk state.
  return radix_sort_plan(n_cap, w->max_fb, c, &w->fb_radix, vals, false);
}

kpa_status learned_sort_launch(const u64* keys_in, const u32* rids_in, u64* keys_out,
                               u32* rids_out, const SegList& sl, const kpa_pwl_model* models,
                               kpa_sort_stats* stats, const LearnedWs& lw, hipStream_t st,
                               const u64* vals_in, u64* vals_out, u32 bucket_log2) {
  KPA_REQUIRE(!vals_in || (vals_out && lw.vals_tmp), KPA_EINVAL,
              "a value column needs an output and a planned buffer");
  const bool vals = vals_in != nullptr;
  u64* vtmp = vals ? lw.vals_tmp : nullptr;
  u64* vout = vals ? vals_out : nullptr;
  const u32 n_seg = sl.n_max;
  if (stats) KPA_CHECK(launch_fill_u64(reinterpret_cast<u64*>(stats), STATS_WORDS, 0, st));
  KPA_CHECK(launch_fill_u32(lw.fb_count, 1, 0, st));
  KPA_CHECK(launch_fill_u32(lw.rl_count, 4, 0, st));
  KPA_CHECK(launch_seg_tiles_list(sl, TILE, lw.ltile_start, st));
  KPA_CHECK(launch_tile_seg(lw.ltile_start, n_seg, sl.n_dev, lw.max_tiles, lw.ltile_seg, st));
  KPA_CHECK(launch_fill_u64(lw.cur_min, n_seg, ~0ull, st));
  KPA_CHECK(launch_fill_u64(lw.cur_max, n_seg, 0ull, st));
  KPA_LAUNCH("learned_minmax", k_seg_minmax, dim3((u32)std::min<u64>(lw.max_tiles, 2048)),
             dim3(BLOCK), 0, st, keys_in, sl, lw.ltile_start, lw.ltile_seg, lw.cur_min,
             lw.cur_max);
  KPA_LAUNCH("learned_setup", k_learned_setup, dim3(std::min<u32>(n_seg, 2048)), dim3(BLOCK), 0,
             st, models, sl, lw.cur_min, lw.cur_max, lw.segm, stats, bucket_log2);
  DigitSortBufs b{keys_in,     rids_in,      keys_out,    rids_out,       lw.keys_tmp,
                  lw.rids_tmp, lw.hist,      lw.seg_mask, lw.ltile_start, lw.status0,
                  lw.status1,  lw.counters,  lw.max_tiles, lw.order,     nullptr,
                  vals_in,     vout,         vtmp};
  KPA_CHECK(digit_sort_launch<LearnedDF>(sl, LearnedDF::Params{lw.segm, models}, b, st));

  KPA_CHECK(launch_seg_tiles_list(sl, FH, lw.ftile_start, st));
  KPA_CHECK(launch_tile_seg(lw.ftile_start, n_seg, sl.n_dev, lw.max_ftiles, lw.ftile_seg, st));
  KPA_CHECK(launch_fill_u32(lw.fn_active, 1, 0, st));
  KPA_LAUNCH("learned_finish_list", k_fin_active,
             dim3((u32)std::min<u64>(ceil_div(lw.max_ftiles, BLOCK), 4096)), dim3(BLOCK), 0, st,
             keys_out, sl, lw.ftile_start, lw.ftile_seg, lw.segm, (u32)lw.max_ftiles, lw.fedge,
             lw.factive, lw.fn_active);
  if (vals)
    KPA_LAUNCH("learned_finish", k_learned_finish<true>, dim3((u32)lw.max_ftiles),
               dim3(FIN_THREADS), 0, st, keys_out, rids_out, vout, sl, lw.ftile_start, lw.fedge,
               lw.segm, lw.factive,
               lw.fn_active, lw.fb_lo, lw.fb_hi, lw.fb_seg, lw.fb_count, lw.max_fb, stats);
  else
    KPA_LAUNCH("learned_finish", k_learned_finish<false>, dim3((u32)lw.max_ftiles),
               dim3(FIN_THREADS), 0, st, keys_out, rids_out, vout, sl, lw.ftile_start, lw.fedge,
               lw.segm, lw.factive,
               lw.fn_active, lw.fb_lo, lw.fb_hi, lw.fb_seg, lw.fb_count, lw.max_fb, stats);

  // Pivot rounds over the oversize chunks: round 0 reads the finishing pass's
  // list, round 1 the parts round 0 left over; small parts collect in one list.
  const u64* lo_in[2] = {lw.fb_lo, lw.rl_lo[0]};
  const u64* hi_in[2] = {lw.fb_hi, lw.rl_hi[0]};
  const u32* cnt_in[2] = {lw.fb_count, lw.rl_count + 0};
  const u32* seg_in[2] = {lw.fb_seg, lw.rl_seg[0]};
  for (int r = 0; r < 2; ++r) {
    const SegList fl{lo_in[r], hi_in[r], cnt_in[r], lw.max_fb};
    KPA_LAUNCH("pivot_select", k_fb_pivot, dim3(1024), dim3(BLOCK), 0, st, keys_out, fl, lw.pivot,
               lw.cnt3);
    KPA_CHECK(launch_seg_tiles_list(fl, TILE, lw.fb_tile_start, st));
    KPA_CHECK(launch_tile_seg(lw.fb_tile_start, lw.max_fb, cnt_in[r],
                              max_tiles(lw.n_cap, lw.max_fb, TILE), lw.fb_tile_seg, st));
    KPA_LAUNCH("pivot_count", k_fb_count, dim3(2048), dim3(BLOCK), 0, st, keys_out, fl,
               lw.fb_tile_start, lw.fb_tile_seg, lw.pivot, lw.cnt3, lw.t_lt, lw.t_eq,
               lw.t_eqbits);
    KPA_LAUNCH("pivot_plan", k_fb_plan, dim3(64), dim3(BLOCK), 0, st, fl, seg_in[r], lw.cnt3,
               lw.p_mask, lw.sm_lo, lw.sm_hi, lw.sm_seg, lw.rl_count + 2, 6 * lw.max_fb,
               lw.rl_lo[r], lw.rl_hi[r], lw.rl_seg[r], lw.rl_count + r, lw.max_fb,
               r == 0 ? stats : nullptr);
    KPA_LAUNCH("pivot_prefix", k_fb_tscan, dim3(1024), dim3(1024), 0, st, fl, lw.fb_tile_start,
               lw.p_mask, lw.t_lt, lw.t_eq);
    KPA_LAUNCH("pivot_move", k_fb_move, dim3(2048), dim3(BLOCK), 0, st, keys_out, rids_out, fl,
               lw.fb_tile_start, lw.fb_tile_seg, lw.pivot, lw.cnt3, lw.p_mask, lw.t_lt, lw.t_eq,
               lw.t_eqbits, lw.keys_tmp, lw.rids_tmp, vout, vtmp);
    KPA_LAUNCH("pivot_back", k_fb_back, dim3(2048), dim3(BLOCK), 0, st, keys_out, rids_out, fl,
               lw.fb_tile_start, lw.fb_tile_seg, lw.pivot, lw.cnt3, lw.p_mask, lw.t_eqbits,
               lw.keys_tmp, lw.rids_tmp, vout, vtmp);
  }
  if (vals)
    KPA_LAUNCH("lds_sort_ranges", k_lds_sort_ranges<true>, dim3(2048), dim3(FIN_THREADS), 0, st,
               keys_out, rids_out, vout, lw.sm_lo, lw.sm_hi, lw.sm_seg, lw.segm, lw.rl_count + 2,
               6 * lw.max_fb);
  else
    KPA_LAUNCH("lds_sort_ranges", k_lds_sort_ranges<false>, dim3(2048), dim3(FIN_THREADS), 0, st,
               keys_out, rids_out, vout, lw.sm_lo, lw.sm_hi, lw.sm_seg, lw.segm, lw.rl_count + 2,
               6 * lw.max_fb);

  // What two rounds did not resolve goes through the radix path.
  const SegList rl{lw.rl_lo[1], lw.rl_hi[1], lw.rl_count + 1, lw.max_fb};
  // in place, with the scatter passes' ping-pong buffers (free by now) as
  // scratch
  return radix_sort_inplace(keys_out, rids_out, vout, rl, lw.fb_radix, lw.keys_tmp, lw.rids_tmp,
                            vtmp, st, stats_unsupported(stats));
}

}  // namespace kpa
