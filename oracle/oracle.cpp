// CPU ORACLE for the KPA grouping path -- TEST INFRASTRUCTURE ONLY.
//
// Plain, slow, obviously correct definitions of what each step computes,
// written from StreamBox-HBM (ASPLOS'19): Sec. 4.1 (KPA = resident key plus a
// pointer to the full record), Table 2 (Extract, Materialize, Sort, Merge,
// Join, Partition, Keyed and unkeyed reduction, Select, KeySwap), Sec. 4.2
// "Compound Operators" (windowing as a partition on the timestamp column, with
// fixed or sliding windows; keyed aggregation; temporal join), Sec. 4.3 (in-
// place key update with write-back; Materialize coalesced with Extract) and
// the benchmark list of Sec. 6 (top-k / sum / median / average / unique count
// per key, average of a window, temporal join, windowed filter).
//
// Only tests, the smoke check and the benchmark's CPU-baseline leg may load
// this library.  It shares no source, header or helper with the GPU library;
// it restates the row byte layout on its own.
//
// Conventions (the readings of the paper used throughout):
//  * a pointer is a row index ("rid") into the stream's arena of fixed-size rows;
//  * keys are unsigned 64-bit and compared as unsigned;
//  * Sort is stable: equal keys keep their input order (for KPAs produced by
//    Extract/Partition that is ascending rid);
//  * Merge is stable: on equal keys every element of the first input comes
//    before every element of the second;
//  * windows are half-open [origin + w*W, origin + (w+1)*W); timestamps outside
//    [origin, origin + n_win*W) are counted and excluded;
//  * sums and products wrap modulo 2^64; the median of an even-sized group is
//    the lower one, v[(n-1)/2] of the ascending values.
//
// Every function returns 0 on success and a negative value on bad arguments.

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <map>
#include <thread>
#include <utility>
#include <vector>

typedef uint64_t u64;
typedef uint32_t u32;

static u64 load_le(const unsigned char* p, int width) {
  u64 v = 0;
  for (int b = width - 1; b >= 0; --b) v = (v << 8) | p[b];
  return v;
}

static const unsigned char* row_at(const void* rows, u64 rid, int row_bytes) {
  return static_cast<const unsigned char*>(rows) + rid * (u64)row_bytes;
}

struct Agg {
  u64 cnt = 0, sum = 0, max = 0;
};

extern "C" {

// Extract + Partition on the timestamp column (Table 2; Sec. 4.2 "Windowing"):
// for every row in arrival order whose timestamp falls in window w, append
// (key, rid_base + row) to window w.  win_off has n_win + 1 entries.
int orc_partition(const void* rows, u64 n, int row_bytes, int key_off, int ts_off, int ts_w,
                  u64 win_len, u64 origin, u32 n_win, u64 rid_base, u64* out_keys, u32* out_rids,
                  u64* out_win_off, u64* out_oob) {
  if (win_len == 0 || (ts_w != 4 && ts_w != 8)) return -1;
  std::vector<std::vector<std::pair<u64, u32>>> win(n_win);
  u64 oob = 0;
  for (u64 i = 0; i < n; ++i) {
    const unsigned char* r = row_at(rows, i, row_bytes);
    u64 ts = load_le(r + ts_off, ts_w);
    if (ts < origin || (ts - origin) / win_len >= n_win) {
      ++oob;
      continue;
    }
    u64 w = (ts - origin) / win_len;
    win[w].push_back({load_le(r + key_off, 8), (u32)(rid_base + i)});
  }
  u64 pos = 0;
  for (u32 w = 0; w < n_win; ++w) {
    out_win_off[w] = pos;
    for (auto& e : win[w]) {
      out_keys[pos] = e.first;
      out_rids[pos] = e.second;
      ++pos;
    }
  }
  out_win_off[n_win] = pos;
  *out_oob = oob;
  return 0;
}

// Extract (Table 2): the key column plus pointers, in arrival order.
int orc_extract(const void* rows, u64 n, int row_bytes, int key_off, u64 rid_base, u64* out_keys,
                u32* out_rids) {
  for (u64 i = 0; i < n; ++i) {
    out_keys[i] = load_le(row_at(rows, i, row_bytes) + key_off, 8);
    out_rids[i] = (u32)(rid_base + i);
  }
  return 0;
}

// Sort (Table 2): stable sort of (key, pointer) pairs by resident key.
int orc_sort(const u64* keys, const u32* rids, u64 n, u64* out_keys, u32* out_rids) {
  std::vector<std::pair<u64, u32>> v(n);
  for (u64 i = 0; i < n; ++i) v[i] = {keys[i], rids[i]};
  std::stable_sort(v.begin(), v.end(),
                   [](const std::pair<u64, u32>& a, const std::pair<u64, u32>& b) {
                     return a.first < b.first;
                   });
  for (u64 i = 0; i < n; ++i) {
    out_keys[i] = v[i].first;
    out_rids[i] = v[i].second;
  }
  return 0;
}

// Sort each segment [seg_off[s], seg_off[s+1]) on its own.
int orc_sort_segmented(const u64* keys, const u32* rids, const u64* seg_off, u32 n_seg,
                       u64* out_keys, u32* out_rids) {
  for (u32 s = 0; s < n_seg; ++s) {
    u64 a = seg_off[s], b = seg_off[s + 1];
    if (b < a) return -1;
    orc_sort(keys + a, rids + a, b - a, out_keys + a, out_rids + a);
  }
  return 0;
}

// Merge (Table 2): two sorted KPAs into one; ties take the first input first.
int orc_merge(const u64* ak, const u32* ar, u64 na, const u64* bk, const u32* br, u64 nb,
              u64* out_keys, u32* out_rids) {
  std::vector<std::pair<u64, u32>> a(na), b(nb), o(na + nb);
  for (u64 i = 0; i < na; ++i) a[i] = {ak[i], ar[i]};
  for (u64 i = 0; i < nb; ++i) b[i] = {bk[i], br[i]};
  std::merge(a.begin(), a.end(), b.begin(), b.end(), o.begin(),
             [](const std::pair<u64, u32>& x, const std::pair<u64, u32>& y) {
               return x.first < y.first;
             });
  for (u64 i = 0; i < na + nb; ++i) {
    out_keys[i] = o[i].first;
    out_rids[i] = o[i].second;
  }
  return 0;
}

// Keyed reduction (Table 2; Sec. 4.2 "Keyed Aggregation"): for every distinct
// resident key, count, sum (mod 2^64) and max of the value column of the rows
// its pointers reach.  Output in ascending key order.  Input order is free.
int orc_reduce_by_key(const u64* keys, const u32* rids, u64 n, const void* rows, int row_bytes,
                      int val_off, int val_w, u64* out_gkey, u64* out_cnt, u64* out_sum,
                      u64* out_max, u64* out_ngroups) {
  if (val_w != 4 && val_w != 8) return -1;
  std::map<u64, Agg> m;
  for (u64 i = 0; i < n; ++i) {
    u64 v = load_le(row_at(rows, rids[i], row_bytes) + val_off, val_w);
    Agg& a = m[keys[i]];
    a.cnt += 1;
    a.sum += v;
    if (v > a.max) a.max = v;
  }
  u64 g = 0;
  for (auto& kv : m) {
    out_gkey[g] = kv.first;
    if (out_cnt) out_cnt[g] = kv.second.cnt;
    if (out_sum) out_sum[g] = kv.second.sum;
    if (out_max) out_max[g] = kv.second.max;
    ++g;
  }
  *out_ngroups = g;
  return 0;
}

// Top-k groups by sum: descending sum, ascending key among equal sums.
int orc_topk_by_sum(const u64* gkey, const u64* gsum, u64 g, u32 k, u64* out_key, u64* out_sum,
                    u32* out_n) {
  std::vector<std::pair<u64, u64>> v(g);  // (sum, key)
  for (u64 i = 0; i < g; ++i) v[i] = {gsum[i], gkey[i]};
  u64 kk = std::min<u64>(k, g);
  std::partial_sort(v.begin(), v.begin() + kk, v.end(),
                    [](const std::pair<u64, u64>& a, const std::pair<u64, u64>& b) {
                      if (a.first != b.first) return a.first > b.first;
                      return a.second < b.second;
                    });
  for (u64 i = 0; i < kk; ++i) {
    out_key[i] = v[i].second;
    out_sum[i] = v[i].first;
  }
  *out_n = (u32)kk;
  return 0;
}

// Median per key (Sec. 6 "Windowed Median Per Key"; percentile-by-key via sort
// and reduction, Sec. 4.2): lower median of each key's values.
int orc_median_by_key(const u64* keys, const u32* rids, u64 n, const void* rows, int row_bytes,
                      int val_off, int val_w, u64* out_gkey, u64* out_med, u64* out_ngroups) {
  if (val_w != 4 && val_w != 8) return -1;
  std::map<u64, std::vector<u64>> m;
  for (u64 i = 0; i < n; ++i)
    m[keys[i]].push_back(load_le(row_at(rows, rids[i], row_bytes) + val_off, val_w));
  u64 g = 0;
  for (auto& kv : m) {
    std::vector<u64>& v = kv.second;
    size_t mid = (v.size() - 1) / 2;
    std::nth_element(v.begin(), v.begin() + mid, v.end());
    out_gkey[g] = kv.first;
    out_med[g] = v[mid];
    ++g;
  }
  *out_ngroups = g;
  return 0;
}

// Join (Table 2; Sec. 4.2 "Temporal Join"): every pair (l, r) of the two
// KPAs with equal keys.  count = number of pairs, sumprod = sum over pairs of
// val_l * val_r (mod 2^64), evaluated pair by pair.  When out_pairs is given,
// the first min(total, cap) pairs in (key, ridL, ridR) order are written as
// three u64 words each.  out_npairs receives the total.
int orc_join(const u64* lk, const u32* lr, u64 nl, const u64* rk, const u32* rr, u64 nr,
             const void* rows_l, const void* rows_r, int row_bytes, int val_off, int val_w,
             u64* out_count, u64* out_sumprod, u64* out_pairs, u64 cap, u64* out_npairs) {
  if (val_w != 4 && val_w != 8) return -1;
  std::map<u64, std::vector<std::pair<u32, u64>>> L, R;  // key -> (rid, val)
  for (u64 i = 0; i < nl; ++i)
    L[lk[i]].push_back({lr[i], load_le(row_at(rows_l, lr[i], row_bytes) + val_off, val_w)});
  for (u64 i = 0; i < nr; ++i)
    R[rk[i]].push_back({rr[i], load_le(row_at(rows_r, rr[i], row_bytes) + val_off, val_w)});
  u64 count = 0, sumprod = 0, np = 0;
  for (auto& kv : L) {
    auto it = R.find(kv.first);
    if (it == R.end()) continue;
    std::vector<std::pair<u32, u64>> a = kv.second, b = it->second;
    std::sort(a.begin(), a.end());
    std::sort(b.begin(), b.end());
    for (auto& x : a)
      for (auto& y : b) {
        count += 1;
        sumprod += x.second * y.second;
        if (out_pairs && np < cap) {
          out_pairs[3 * np + 0] = kv.first;
          out_pairs[3 * np + 1] = x.first;
          out_pairs[3 * np + 2] = y.first;
        }
        ++np;
      }
  }
  *out_count = count;
  *out_sumprod = sumprod;
  if (out_npairs) *out_npairs = np;
  return 0;
}

// Materialize (Table 2): the full rows in KPA order.
int orc_materialize(const u32* rids, u64 n, const void* rows, int row_bytes, void* out_rows) {
  unsigned char* o = static_cast<unsigned char*>(out_rows);
  for (u64 i = 0; i < n; ++i) std::memcpy(o + i * row_bytes, row_at(rows, rids[i], row_bytes), row_bytes);
  return 0;
}

// Piecewise-linear CDF model fit from a sorted KPA.  kmin/kmax are the first
// and last keys; boundary j (0..n_seg) is kmin + floor(j * (kmax - kmin) / n_seg)
// and knot j is (number of keys strictly below boundary j) / n, rounded once
// from the exact ratio to float32.
int orc_pwl_fit(const u64* sorted_keys, u64 n, u32 n_seg, u64* out_kmin, u64* out_kmax,
                float* out_knots) {
  if (n == 0 || n_seg == 0) return -1;
  u64 kmin = sorted_keys[0], kmax = sorted_keys[n - 1];
  u64 span = kmax - kmin;
  for (u32 j = 0; j <= n_seg; ++j) {
    unsigned __int128 off = (unsigned __int128)span * j / n_seg;
    u64 b = kmin + (u64)off;
    u64 below = (u64)(std::lower_bound(sorted_keys, sorted_keys + n, b) - sorted_keys);
    out_knots[j] = (float)((double)below / (double)n);
  }
  *out_kmin = kmin;
  *out_kmax = kmax;
  return 0;
}

// One full window of the windowed keyed aggregation (for the CPU baseline):
// partition by timestamp, then per window an ordered map of count/sum/max and
// the top-k keys by sum.  One std::thread per window, at most n_threads.
// out_groups[w] receives the number of groups of window w; out_top (n_win*k
// (key, sum) pairs) the top-k lists.
int orc_window_aggregate(const void* rows, u64 n, int row_bytes, int key_off, int val_off,
                         int val_w, int ts_off, int ts_w, u64 win_len, u64 origin, u32 n_win,
                         u32 k, int n_threads, u64* out_groups, u64* out_top_key,
                         u64* out_top_sum, u64* out_checksum) {
  if (win_len == 0 || n_threads < 1) return -1;
  std::vector<std::map<u64, Agg>> maps(n_win);
  auto work = [&](u32 w0, u32 w1) {
    for (u64 i = 0; i < n; ++i) {
      const unsigned char* r = row_at(rows, i, row_bytes);
      u64 ts = load_le(r + ts_off, ts_w);
      if (ts < origin) continue;
      u64 w = (ts - origin) / win_len;
      if (w < w0 || w >= w1) continue;
      u64 v = load_le(r + val_off, val_w);
      Agg& a = maps[w][load_le(r + key_off, 8)];
      a.cnt += 1;
      a.sum += v;
      if (v > a.max) a.max = v;
    }
  };
  u32 nt = std::min<u32>((u32)n_threads, n_win ? n_win : 1);
  std::vector<std::thread> th;
  u32 per = (n_win + nt - 1) / nt;
  for (u32 t = 0; t < nt; ++t) {
    u32 a = t * per, b = std::min<u32>(n_win, a + per);
    if (a < b) th.emplace_back(work, a, b);
  }
  for (auto& t : th) t.join();
  u64 cs = 0;
  for (u32 w = 0; w < n_win; ++w) {
    out_groups[w] = maps[w].size();
    std::vector<u64> gk, gs;
    for (auto& kv : maps[w]) {
      gk.push_back(kv.first);
      gs.push_back(kv.second.sum);
      cs += kv.first * 31 + kv.second.cnt * 7 + kv.second.sum * 3 + kv.second.max;
    }
    u32 got = 0;
    orc_topk_by_sum(gk.data(), gs.data(), gk.size(), k, out_top_key + (u64)w * k,
                    out_top_sum + (u64)w * k, &got);
    for (u32 i = got; i < k; ++i) out_top_key[(u64)w * k + i] = out_top_sum[(u64)w * k + i] = 0;
  }
  *out_checksum = cs;
  return 0;
}

// ---------------------------------------------------------------------------
// Single-pass benchmarks of Sec. 6 (benchmark list) and the remaining Table 2
// primitives.

// TopK Per Key (Sec. 6, benchmark 1): for every distinct key, its k largest
// values in descending order (a multiset: equal values repeat).  Output in
// ascending key order: out_gkey[g], out_gcnt[g] (entries of the key),
// out_tn[g] = min(k, count) and out_topv[g*k + j], j < out_tn[g] (the rest of
// the row is set to 0).
int orc_topk_per_key(const u64* keys, const u32* rids, u64 n, const void* rows, int row_bytes,
                     int val_off, int val_w, u32 k, u64* out_gkey, u64* out_gcnt, u32* out_tn,
                     u64* out_topv, u64* out_ngroups) {
  if ((val_w != 4 && val_w != 8) || k == 0) return -1;
  std::map<u64, std::vector<u64>> m;
  for (u64 i = 0; i < n; ++i)
    m[keys[i]].push_back(load_le(row_at(rows, rids[i], row_bytes) + val_off, val_w));
  u64 g = 0;
  for (auto& kv : m) {
    std::vector<u64>& v = kv.second;
    std::sort(v.begin(), v.end(), [](u64 a, u64 b) { return a > b; });
    u32 t = (u32)std::min<u64>(k, v.size());
    out_gkey[g] = kv.first;
    out_gcnt[g] = v.size();
    out_tn[g] = t;
    for (u32 j = 0; j < k; ++j) out_topv[g * k + j] = j < t ? v[j] : 0;
    ++g;
  }
  *out_ngroups = g;
  return 0;
}

// Unique Count Per Key (Sec. 6, benchmark 6): for every distinct key, the
// number of distinct values among its records.  Ascending key order.
int orc_unique_count_by_key(const u64* keys, const u32* rids, u64 n, const void* rows,
                            int row_bytes, int val_off, int val_w, u64* out_gkey, u64* out_uniq,
                            u64* out_ngroups) {
  if (val_w != 4 && val_w != 8) return -1;
  std::map<u64, std::vector<u64>> m;
  for (u64 i = 0; i < n; ++i)
    m[keys[i]].push_back(load_le(row_at(rows, rids[i], row_bytes) + val_off, val_w));
  u64 g = 0;
  for (auto& kv : m) {
    std::vector<u64>& v = kv.second;
    std::sort(v.begin(), v.end());
    out_gkey[g] = kv.first;
    out_uniq[g] = (u64)(std::unique(v.begin(), v.end()) - v.begin());
    ++g;
  }
  *out_ngroups = g;
  return 0;
}

// Unkeyed reduction over windows (Table 2 "Unkeyed reduction"; Sec. 6,
// benchmark 5 "Windowed Average All"): for each window w of the rows (window
// rule as orc_partition), the number of rows, the exact sum of their values as
// a 128-bit integer (out_sum_lo + 2^64 * out_sum_hi) and the largest value.
// The average is sum / count (left to the caller, so that it stays exact).
int orc_reduce_all_windows(const void* rows, u64 n, int row_bytes, int val_off, int val_w,
                           int ts_off, int ts_w, u64 win_len, u64 origin, u32 n_win, u64* out_cnt,
                           u64* out_sum_lo, u64* out_sum_hi, u64* out_max, u64* out_oob) {
  if (win_len == 0 || (ts_w != 4 && ts_w != 8) || (val_w != 4 && val_w != 8)) return -1;
  std::vector<unsigned __int128> sum(n_win, 0);
  for (u32 w = 0; w < n_win; ++w) out_cnt[w] = out_max[w] = 0;
  u64 oob = 0;
  for (u64 i = 0; i < n; ++i) {
    const unsigned char* r = row_at(rows, i, row_bytes);
    u64 ts = load_le(r + ts_off, ts_w);
    if (ts < origin || (ts - origin) / win_len >= n_win) {
      ++oob;
      continue;
    }
    u64 w = (ts - origin) / win_len;
    u64 v = load_le(r + val_off, val_w);
    out_cnt[w] += 1;
    sum[w] += v;
    if (v > out_max[w]) out_max[w] = v;
  }
  for (u32 w = 0; w < n_win; ++w) {
    out_sum_lo[w] = (u64)sum[w];
    out_sum_hi[w] = (u64)(sum[w] >> 64);
  }
  *out_oob = oob;
  return 0;
}

// Select (Table 2: keep the pairs that pass a predicate, in their order).  For
// every segment s of a KPA, entry i passes when x_i * den[s] <op> num[s], with
// x_i the resident key (column 0) or the value of its row (column 1),
// num[s] = num_lo[s] + 2^64 * num_hi[s] and the product taken exactly.
// op: 0 '>', 1 '>=', 2 '<', 3 '<=', 4 '==', 5 '!='.  Survivors are written
// back to back, segment after segment, with out_seg_off (n_seg + 1).
int orc_select(const u64* keys, const u32* rids, const u64* seg_off, u32 n_seg, const void* rows,
               int row_bytes, int val_off, int val_w, int column, int op, const u64* num_lo,
               const u64* num_hi, const u64* den, u64* out_keys, u32* out_rids,
               u64* out_seg_off) {
  if (column != 0 && column != 1) return -1;
  if (column == 1 && val_w != 4 && val_w != 8) return -1;
  if (op < 0 || op > 5) return -1;
  u64 pos = 0;
  for (u32 s = 0; s < n_seg; ++s) {
    out_seg_off[s] = pos;
    unsigned __int128 rhs = ((unsigned __int128)num_hi[s] << 64) | num_lo[s];
    for (u64 i = seg_off[s]; i < seg_off[s + 1]; ++i) {
      u64 x = column == 0 ? keys[i] : load_le(row_at(rows, rids[i], row_bytes) + val_off, val_w);
      unsigned __int128 lhs = (unsigned __int128)x * den[s];
      bool keep = op == 0 ? lhs > rhs : op == 1 ? lhs >= rhs : op == 2 ? lhs < rhs
                : op == 3 ? lhs <= rhs : op == 4 ? lhs == rhs : lhs != rhs;
      if (keep) {
        out_keys[pos] = keys[i];
        out_rids[pos] = rids[i];
        ++pos;
      }
    }
  }
  out_seg_off[n_seg] = pos;
  return 0;
}

// Windowed Filter (Sec. 6, benchmark 8): the average of stream A's values in
// window w filters the keys of stream B in the same window.  B's row passes
// when its key is above that average, key > sum_A(w) / count_A(w), decided
// exactly as key * count_A(w) > sum_A(w); a window of A without rows lets
// nothing pass.  Output: B's passing (key, rid) per window in arrival order
// (window rule as orc_partition), with out_win_off (n_win + 1).
int orc_window_filter(const void* rows_a, u64 na, const void* rows_b, u64 nb, int row_bytes,
                      int key_off, int val_off, int val_w, int ts_off, int ts_w, u64 win_len,
                      u64 origin, u32 n_win, u64 rid_base_b, u64* out_keys, u32* out_rids,
                      u64* out_win_off) {
  if (win_len == 0 || (ts_w != 4 && ts_w != 8) || (val_w != 4 && val_w != 8)) return -1;
  std::vector<u64> cnt(n_win, 0);
  std::vector<unsigned __int128> sum(n_win, 0);
  for (u64 i = 0; i < na; ++i) {
    const unsigned char* r = row_at(rows_a, i, row_bytes);
    u64 ts = load_le(r + ts_off, ts_w);
    if (ts < origin || (ts - origin) / win_len >= n_win) continue;
    u64 w = (ts - origin) / win_len;
    cnt[w] += 1;
    sum[w] += load_le(r + val_off, val_w);
  }
  std::vector<std::vector<std::pair<u64, u32>>> win(n_win);
  for (u64 i = 0; i < nb; ++i) {
    const unsigned char* r = row_at(rows_b, i, row_bytes);
    u64 ts = load_le(r + ts_off, ts_w);
    if (ts < origin || (ts - origin) / win_len >= n_win) continue;
    u64 w = (ts - origin) / win_len;
    u64 key = load_le(r + key_off, 8);
    if (cnt[w] > 0 && (unsigned __int128)key * cnt[w] > sum[w])
      win[w].push_back({key, (u32)(rid_base_b + i)});
  }
  u64 pos = 0;
  for (u32 w = 0; w < n_win; ++w) {
    out_win_off[w] = pos;
    for (auto& e : win[w]) {
      out_keys[pos] = e.first;
      out_rids[pos] = e.second;
      ++pos;
    }
  }
  out_win_off[n_win] = pos;
  return 0;
}

// KeySwap (Table 2: load a nonresident column and make it the resident key):
// out_keys[i] = the column (col_w = 4 or 8 bytes at col_off, zero-extended)
// of row rids[i].
int orc_keyswap(const u32* rids, u64 n, const void* rows, int row_bytes, int col_off, int col_w,
                u64* out_keys) {
  if (col_w != 4 && col_w != 8) return -1;
  for (u64 i = 0; i < n; ++i) out_keys[i] = load_le(row_at(rows, rids[i], row_bytes) + col_off, col_w);
  return 0;
}

// In-place key update from a key-value table (Sec. 4.3, optimization 2; the
// external join of the pipeline example): every resident key found among the
// table's keys is replaced by the table's value for it; keys not in the table
// are kept and counted in *out_missing.  The table's keys are distinct.
int orc_key_update(u64* keys, u64 n, const u64* tkeys, const u64* tvals, u64 tn,
                   u64* out_missing) {
  std::map<u64, u64> t;
  for (u64 j = 0; j < tn; ++j) t[tkeys[j]] = tvals[j];
  u64 miss = 0;
  for (u64 i = 0; i < n; ++i) {
    auto it = t.find(keys[i]);
    if (it == t.end()) ++miss;
    else keys[i] = it->second;
  }
  *out_missing = miss;
  return 0;
}

// Write-back of resident keys to their rows (Sec. 4.3, optimization 2): the
// column at col_off (8 bytes) of row rids[i] becomes keys[i].  rids are
// distinct.
int orc_key_writeback(const u64* keys, const u32* rids, u64 n, void* rows, int row_bytes,
                      int col_off) {
  unsigned char* base = static_cast<unsigned char*>(rows);
  for (u64 i = 0; i < n; ++i) {
    unsigned char* p = base + (u64)rids[i] * row_bytes + col_off;
    for (int b = 0; b < 8; ++b) p[b] = (unsigned char)(keys[i] >> (8 * b));
  }
  return 0;
}

// Materialize coalesced with Extract (Sec. 4.3, optimization 1): the rows in
// KPA order (as orc_materialize) and, from those emitted rows, the next KPA on
// the column at key_off: out_keys[i] = that column of output row i, out_rids[i]
// = rid_base + i.
int orc_materialize_extract(const u32* rids, u64 n, const void* rows, int row_bytes, int key_off,
                            u64 rid_base, void* out_rows, u64* out_keys, u32* out_rids) {
  unsigned char* o = static_cast<unsigned char*>(out_rows);
  for (u64 i = 0; i < n; ++i) {
    std::memcpy(o + i * row_bytes, row_at(rows, rids[i], row_bytes), row_bytes);
    out_keys[i] = load_le(o + i * row_bytes + key_off, 8);
    out_rids[i] = (u32)(rid_base + i);
  }
  return 0;
}

// Sliding windows (Sec. 4.2 "Windowing": windows of length win_len that start
// every slide): window w covers [origin + w*slide, origin + w*slide + win_len),
// 0 <= w < n_win, so a row belongs to every window whose range holds its
// timestamp.  Per window, per distinct key (ascending): count, sum (mod 2^64)
// and max of the values.  out_gseg_off (n_win + 1) delimits the windows'
// groups; outputs hold up to cap groups in all.
int orc_sliding_aggregate(const void* rows, u64 n, int row_bytes, int key_off, int val_off,
                          int val_w, int ts_off, int ts_w, u64 win_len, u64 slide, u64 origin,
                          u32 n_win, u64 cap, u64* out_gkey, u64* out_cnt, u64* out_sum,
                          u64* out_max, u64* out_gseg_off) {
  if (win_len == 0 || slide == 0 || (ts_w != 4 && ts_w != 8) || (val_w != 4 && val_w != 8))
    return -1;
  std::vector<std::map<u64, Agg>> maps(n_win);
  for (u64 i = 0; i < n; ++i) {
    const unsigned char* r = row_at(rows, i, row_bytes);
    u64 ts = load_le(r + ts_off, ts_w);
    if (ts < origin) continue;
    u64 key = load_le(r + key_off, 8), v = load_le(r + val_off, val_w);
    for (u32 w = 0; w < n_win; ++w) {
      u64 lo = origin + (u64)w * slide;
      if (ts >= lo && ts - lo < win_len) {
        Agg& a = maps[w][key];
        a.cnt += 1;
        a.sum += v;
        if (v > a.max) a.max = v;
      }
    }
  }
  u64 g = 0;
  for (u32 w = 0; w < n_win; ++w) {
    out_gseg_off[w] = g;
    for (auto& kv : maps[w]) {
      if (g >= cap) return -2;
      out_gkey[g] = kv.first;
      out_cnt[g] = kv.second.cnt;
      out_sum[g] = kv.second.sum;
      out_max[g] = kv.second.max;
      ++g;
    }
  }
  out_gseg_off[n_win] = g;
  return 0;
}

// Grouping on full records without KPAs (the "NoKPA" design of the ablation of
// Sec. 7.3): the rows themselves are ordered by (window, key), stably, so each
// window's rows come out grouped by key in arrival order within a key.  Rows
// whose timestamp lies in no window (window rule as orc_partition) count as
// window n_win and come last.  out_rows holds all n rows; out_win_off (n_win
// + 1) delimits the windows; *out_oob counts the rows after out_win_off[n_win].
int orc_sort_rows_windowed(const void* rows, u64 n, int row_bytes, int key_off, int ts_off,
                           int ts_w, u64 win_len, u64 origin, u32 n_win, void* out_rows,
                           u64* out_win_off, u64* out_oob) {
  if (win_len == 0 || (ts_w != 4 && ts_w != 8)) return -1;
  std::vector<std::pair<std::pair<u64, u64>, u64>> v(n);  // ((window, key), row)
  for (u64 i = 0; i < n; ++i) {
    const unsigned char* r = row_at(rows, i, row_bytes);
    u64 ts = load_le(r + ts_off, ts_w);
    u64 w = (ts < origin || (ts - origin) / win_len >= n_win) ? n_win : (ts - origin) / win_len;
    v[i] = {{w, load_le(r + key_off, 8)}, i};
  }
  std::stable_sort(v.begin(), v.end(),
                   [](const std::pair<std::pair<u64, u64>, u64>& a,
                      const std::pair<std::pair<u64, u64>, u64>& b) { return a.first < b.first; });
  unsigned char* o = static_cast<unsigned char*>(out_rows);
  for (u64 i = 0; i < n; ++i) std::memcpy(o + i * row_bytes, row_at(rows, v[i].second, row_bytes), row_bytes);
  u64 pos = 0;
  for (u32 w = 0; w <= n_win; ++w) {
    out_win_off[w] = pos;
    while (pos < n && v[pos].first.first == w) ++pos;
  }
  *out_oob = n - out_win_off[n_win];
  return 0;
}

}  // extern "C"
