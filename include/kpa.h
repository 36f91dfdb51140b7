/*
 * kpa.h -- C ABI of the Key Pointer Array (KPA) grouping library for AMD
 * Instinct MI355X (gfx950).
 *
 * A KPA (StreamBox-HBM, ASPLOS'19, Sec. 4.1) is a sequence of pairs of one
 * resident key column and a pointer to the full record.  Here the pointer is a
 * 32-bit row index ("rid") into the caller's arena of fixed-size rows, and a
 * KPA is stored as two parallel device arrays: uint64_t keys[n], uint32_t
 * rids[n] (12 bytes per entry).  The calls implement the primitives of the
 * paper's Table 2 (Extract, Partition, Sort, Merge, Join, Keyed reduction,
 * Materialize) and the compound operators of Sec. 4.2 built on them
 * (windowing = partition on the timestamp column; keyed aggregation = sort
 * then per-key reduction; temporal join = sort both sides then one scan).
 *
 * Conventions for every call
 *  - Return value: kpa_status (0 = KPA_OK).  No C++ exception crosses the ABI.
 *    On failure nothing has been enqueued unless the status is KPA_EHIP; the
 *    message is available from kpa_last_error_string() (thread-local).
 *  - Ownership: every array is allocated and owned by the caller.  Arrays named
 *    "device" must be device memory (or host memory mapped for device access)
 *    of the current HIP device.  The stateless calls never allocate: a call
 *    that needs scratch memory takes a workspace pointer (device memory, 256-
 *    byte aligned) and its size; kpa_<op>_workspace_size() reports the size.
 *    Too small a workspace returns KPA_EWORKSPACE.
 *  - Asynchrony: every call enqueues work on `stream` and returns; outputs are
 *    valid once the stream has been synchronized.  Scalar outputs (counts,
 *    sums) are device pointers.  Calls on one stream run in order; calls on
 *    different streams must not share a workspace.
 *  - Alignment: keys/u64 arrays 8-byte aligned, rids 4-byte aligned, row
 *    arenas 16-byte aligned, otherwise KPA_EINVAL.
 *  - Sizes: n = 0 is a valid no-op.  A KPA holds fewer than 2^32 entries
 *    (rids are 32-bit).  A segment that a sort or keyed operation works on
 *    holds fewer than 2^30 entries: a larger sort segment is copied through
 *    unsorted and counted in kpa_sort_stats.unsupported_entries.
 *  - Keys are unsigned 64-bit and compared as unsigned.
 *  - Sums and products wrap modulo 2^64.
 */
#ifndef KPA_H_
#define KPA_H_

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t kpa_status;
enum {
  KPA_OK = 0,
  KPA_EINVAL = -1,       /* bad argument (null pointer, misalignment, bad layout) */
  KPA_EWORKSPACE = -2,   /* workspace too small; *needed bytes written where asked */
  KPA_ECAPACITY = -3,    /* an output exceeds the capacity the caller gave */
  KPA_EBUDGET = -4,      /* serving admission: memory budget exhausted */
  KPA_EUNSUPPORTED = -5, /* size or parameter beyond what the library supports */
  KPA_EHIP = -6,         /* a HIP runtime call failed; see kpa_last_error_string() */
  KPA_ETIMEOUT = -7      /* a wait with a time limit ended before the work did */
};

/* Byte layout of a fixed-size little-endian row ("full record").  The key is a
 * u64 at key_off; value and timestamp are u32 or u64 (width 4 or 8). */
typedef struct kpa_row_layout {
  uint32_t row_bytes; /* multiple of 8, at most 256 */
  uint32_t key_off;   /* 8-byte aligned offset of the u64 key */
  uint32_t val_off;   /* offset of the value column, aligned to val_w */
  uint32_t val_w;     /* 4 or 8 */
  uint32_t ts_off;    /* offset of the event timestamp, aligned to ts_w */
  uint32_t ts_w;      /* 4 or 8 */
} kpa_row_layout;

/* Library version (major*10000 + minor*100 + patch). */
int32_t kpa_version(void);
/* Message of the last failing call on this thread ("" if none). */
const char* kpa_last_error_string(void);
/* The HIP error code behind the last KPA_EHIP status on this thread
 * (hipSuccess if the last failure was not a HIP error). */
int32_t kpa_last_hip_error(void);
/* Sets *out to 1 if the current HIP device is gfx950, else 0. */
kpa_status kpa_device_check(int32_t* out);

/* Per-kernel timing (tracing aid; not part of any primitive).  While enabled,
 * every launch is bracketed by HIP events on its own stream.  enable(1) also
 * clears earlier records.  collect() waits for the recorded events and adds
 * their durations to per-kernel totals; get() returns the number of launches
 * and total milliseconds of one kernel name; names() lists the names seen, comma
 * separated, into buf. */
kpa_status kpa_profile_enable(int32_t on);
kpa_status kpa_profile_collect(void);
kpa_status kpa_profile_get(const char* name, uint64_t* launches, double* total_ms);
kpa_status kpa_profile_names(char* buf, size_t len);

/* ---------------------------------------------------------------------------
 * Extract (Table 2: bundle -> KPA, sequential).  keys[i] = u64 at key_off of
 * row i, rids[i] = rid_base + i.  rows: device, n rows.  out_keys/out_rids:
 * device, n entries each; out_rids may be NULL when the sort that follows
 * takes NULL row ids (then entry i's row id is i).  out_vals (device, n u64,
 * may be NULL): the value
 * column (val_off, zero-extended) of row i, a compact copy a keyed reduction
 * can read as 8-byte rows (see kpa_partition_windows).
 */
kpa_status kpa_extract(const void* rows, uint64_t n, const kpa_row_layout* layout,
                       uint32_t rid_base, uint64_t* out_keys, uint32_t* out_rids,
                       uint64_t* out_vals, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Extract fused with windowing (Sec. 4.2 "Windowing": Partition on the
 * timestamp column with the window length as the range of each partition).
 * Window w holds the rows whose timestamp ts satisfies
 *   win_origin + w*win_len <= ts < win_origin + (w+1)*win_len,  0 <= w < n_win,
 * in arrival order (ascending rid = rid_base + row index).  The windows are
 * written back to back into out_keys/out_rids (device, capacity n each);
 * out_win_off (device, n_win+1 u64) receives the start of each window and the
 * total.  Rows outside all windows are not written; their number goes to
 * *out_oob (device u64).  1 <= n_win <= 256, win_len >= 1, n < 2^32.
 * out_vals (device, n u64, may be NULL): the value column (layout->val_off,
 * zero-extended) of every row in arrival order, out_vals[i] for row i.  It is
 * a compact copy of one nonresident column: a keyed reduction can read its
 * values there (as 8-byte rows) instead of in the full rows.
 */
kpa_status kpa_partition_windows_workspace_size(uint64_t n, uint32_t n_win, size_t* bytes);
kpa_status kpa_partition_windows(const void* rows, uint64_t n, const kpa_row_layout* layout,
                                 uint64_t win_len, uint64_t win_origin, uint32_t n_win,
                                 uint32_t rid_base, uint64_t* out_keys, uint32_t* out_rids,
                                 uint64_t* out_vals, uint64_t* out_win_off, uint64_t* out_oob,
                                 void* ws, size_t ws_bytes, hipStream_t stream);
/* Partition of a KPA whose resident key is the timestamp (Table 2 Partition;
 * the Window operator of the pipeline example partitions KPA(t)): entry i
 * (keys[i], rids[i]) goes to the window of keys[i] (window rule as above),
 * stably; out_keys/out_rids/out_win_off/out_oob as above.  n < 2^32.
 * Workspace: kpa_partition_windows_workspace_size(n, n_win). */
kpa_status kpa_partition_kpa(const uint64_t* keys, const uint32_t* rids, uint64_t n,
                             uint64_t win_len, uint64_t win_origin, uint32_t n_win,
                             uint64_t* out_keys, uint32_t* out_rids, uint64_t* out_win_off,
                             uint64_t* out_oob, void* ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Sort (Table 2: KPA(c) -> KPA(c), sequential access).  Stable sort by key:
 * equal keys keep their input order (for KPAs from Extract/Partition, that is
 * ascending rid).  Segmented form: segment s is [seg_off[s], seg_off[s+1])
 * (seg_off: device, n_seg+1 u64, nondecreasing, seg_off[n_seg] <= n_cap) and
 * is sorted on its own; all segments go through the same launches.  n_cap is
 * a host-side upper bound on seg_off[n_seg] used to size launches.  keys_in
 * must not alias keys_out (likewise rids).  The inputs are not modified.
 * rids_in may be NULL (here and in the batched and _vals forms): entry i's
 * row id is then i, its position in keys_in (what kpa_extract with rid_base
 * 0 writes), and no input row ids are read.
 *
 * algo KPA_SORT_RADIX: least-significant-digit radix sort with 8-bit digits;
 * digits that are constant within a segment are skipped.
 * algo KPA_SORT_LEARNED: a learned-splitter sort.  models (device, one
 * kpa_pwl_model per segment) give a nondecreasing CDF estimate F; each key goes
 * to bucket floor(B*F(key)), buckets are formed by stable scatters and each
 * bucket is finished in on-chip memory.  The knots are used as the shape of
 * the CDF over the segment's own key range: F(key) interpolates the knots at
 * n_seg*(key - min)/(max - min), with min/max the smallest and largest key of
 * a sample of the segment (the first 256 keys of every 4096-entry tile; keys
 * outside [min, max] go to the first or last bucket), so that a model fitted
 * on an earlier window still applies when the keys have moved by an offset;
 * the model's kmin/kmax record the range it was fitted on.  Buckets too large for that, or whose
 * order the model would break, are re-sorted by the radix path.  The model
 * affects only speed: the output equals the radix sort's, byte for byte.
 * stats (device, may be NULL) receives counters of the learned path.
 */
typedef enum kpa_sort_algo { KPA_SORT_RADIX = 0, KPA_SORT_LEARNED = 1 } kpa_sort_algo;

#define KPA_PWL_MAX_SEG 1024
/* Piecewise-linear CDF model with n_seg equal-width segments over
 * [kmin, kmax]; knots[j] = estimate of F at kmin + floor(j*(kmax-kmin)/n_seg).
 * F(key) = 0 below kmin, 1 above kmax, linear between knots (clamped to the
 * segment's knots so that F never decreases).  Lives in device memory. */
typedef struct kpa_pwl_model {
  uint64_t kmin;
  uint64_t kmax;
  uint32_t n_seg; /* 1..KPA_PWL_MAX_SEG; 0 marks an empty (unusable) model */
  uint32_t reserved;
  float knots[KPA_PWL_MAX_SEG + 1];
  float pad[3];
} kpa_pwl_model;

typedef struct kpa_sort_stats {
  uint64_t n_buckets;          /* buckets formed by the learned path */
  uint64_t finished_on_chip;   /* entries sorted in on-chip memory */
  uint64_t equal_key_entries;  /* entries in single-key buckets (no sort needed) */
  uint64_t fallback_entries;   /* entries re-sorted by the radix path */
  uint64_t fallback_buckets;   /* buckets re-sorted by the radix path */
  uint64_t order_violations;   /* buckets whose key range overlapped a neighbour */
  uint64_t unsupported_entries; /* entries of segments of 2^30 or more entries: copied
                                   through unsorted (the caller must check this) */
} kpa_sort_stats;

kpa_status kpa_sort_workspace_size(uint64_t n_cap, uint32_t n_seg, kpa_sort_algo algo,
                                   size_t* bytes);
kpa_status kpa_sort_segmented(const uint64_t* keys_in, const uint32_t* rids_in,
                              uint64_t* keys_out, uint32_t* rids_out, const uint64_t* seg_off,
                              uint32_t n_seg, uint64_t n_cap, kpa_sort_algo algo,
                              const kpa_pwl_model* models, kpa_sort_stats* stats, void* ws,
                              size_t ws_bytes, hipStream_t stream);
/* One segment of n entries (n known on the host). */
kpa_status kpa_sort(const uint64_t* keys_in, const uint32_t* rids_in, uint64_t n,
                    uint64_t* keys_out, uint32_t* rids_out, kpa_sort_algo algo,
                    const kpa_pwl_model* model, kpa_sort_stats* stats, void* ws, size_t ws_bytes,
                    hipStream_t stream);
/* The same sort with one 8-byte column carried beside the KPA: vals_in[i]
 * belongs to entry i and vals_out receives it at that entry's sorted
 * position (keys_out and rids_out exactly as kpa_sort_segmented writes them).
 * A keyed reduction over that column then reads it in KPA order (row ids
 * NULL in kpa_reduce_by_key) instead of following each row id to its record
 * (Sec. 4.2 keyed aggregation dereferences one column per entry).  Costs 16
 * bytes of traffic per entry and pass more than the KPA alone.  vals_in and
 * vals_out: device, n_cap each, 8-byte aligned, not aliasing each other or
 * the KPA arrays.  Workspace from kpa_sort_vals_workspace_size (larger than
 * kpa_sort_workspace_size by the column's ping-pong buffers). */
kpa_status kpa_sort_vals_workspace_size(uint64_t n_cap, uint32_t n_seg, kpa_sort_algo algo,
                                        size_t* bytes);
kpa_status kpa_sort_segmented_vals(const uint64_t* keys_in, const uint32_t* rids_in,
                                   const uint64_t* vals_in, uint64_t* keys_out,
                                   uint32_t* rids_out, uint64_t* vals_out,
                                   const uint64_t* seg_off, uint32_t n_seg, uint64_t n_cap,
                                   kpa_sort_algo algo, const kpa_pwl_model* models,
                                   kpa_sort_stats* stats, void* ws, size_t ws_bytes,
                                   hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Batched sort of many uneven segments (the windows of many substreams, all
 * in flight at once; the paper gets its parallelism from many bundles and
 * windows processed concurrently and out of order, Sec. 3).  Same contract
 * as kpa_sort_segmented (stable; the output equals it byte for byte), with
 * the segments split by size:
 *   n <= small_cap           one workgroup sorts the segment in LDS;
 *   small_cap < n <= mid_cap one workgroup runs the radix passes through
 *                            device memory, with no cross-workgroup traffic;
 *   n > mid_cap              the multi-workgroup path of large_algo
 *                            (KPA_SORT_RADIX or KPA_SORT_LEARNED; models as
 *                            in kpa_sort_segmented, used for these segments).
 * A device-side work table (largest segments first) is drained by one
 * persistent kernel; segment sizes are read from seg_off on the device only,
 * so a captured graph of this call serves any segmentation with the same
 * n_seg and n_cap.  small_cap <= 4096, small_cap <= mid_cap < 2^30; grid = 0
 * sizes the persistent kernel to the workgroups resident at once.
 * bucket_log2 (learned large path): the bucket count of a segment of n
 * entries is the power of two nearest above n / 2^bucket_log2, in 6..12;
 * 0: 9 (512-entry buckets). */
typedef struct kpa_batch_config {
  uint32_t small_cap;
  uint32_t mid_cap;
  uint32_t grid;
  uint32_t large_algo; /* a kpa_sort_algo */
  uint32_t bucket_log2;
} kpa_batch_config;

/* small_cap 4096, mid_cap 65536, grid 0, bucket_log2 0. */
kpa_status kpa_batch_config_default(kpa_sort_algo large_algo, kpa_batch_config* cfg);
kpa_status kpa_batch_sort_workspace_size(uint64_t n_cap, uint32_t n_seg,
                                         const kpa_batch_config* cfg, size_t* bytes);
kpa_status kpa_batch_sort(const uint64_t* keys_in, const uint32_t* rids_in, uint64_t* keys_out,
                          uint32_t* rids_out, const uint64_t* seg_off, uint32_t n_seg,
                          uint64_t n_cap, const kpa_batch_config* cfg,
                          const kpa_pwl_model* models, kpa_sort_stats* stats, void* ws,
                          size_t ws_bytes, hipStream_t stream);
/* kpa_batch_sort with one 8-byte column carried beside the KPA (as
 * kpa_sort_segmented_vals: vals_out[j] is the value of the entry sorted to
 * position j).  Workspace from kpa_batch_sort_vals_workspace_size. */
kpa_status kpa_batch_sort_vals_workspace_size(uint64_t n_cap, uint32_t n_seg,
                                              const kpa_batch_config* cfg, size_t* bytes);
kpa_status kpa_batch_sort_vals(const uint64_t* keys_in, const uint32_t* rids_in,
                               const uint64_t* vals_in, uint64_t* keys_out, uint32_t* rids_out,
                               uint64_t* vals_out, const uint64_t* seg_off, uint32_t n_seg,
                               uint64_t n_cap, const kpa_batch_config* cfg,
                               const kpa_pwl_model* models, kpa_sort_stats* stats, void* ws,
                               size_t ws_bytes, hipStream_t stream);
/* Autotuner: times kpa_batch_sort on the given batch (one warm-up and `reps`
 * timed runs per candidate) over the class boundaries small_cap in {1024,
 * 2048, 4096} and mid_cap in {small_cap, 2^14, 2^16, 2^18}, then, for the
 * learned large path, the bucket size 2^bucket_log2 in {256, 512, 1024} at the
 * best boundaries, and returns the fastest configuration in *best (its mean
 * time in *best_ms, may be NULL).
 * cache_path (host file, may be NULL): a text file of earlier results keyed by
 * the batch's signature (segment count, capacity, large_algo and a coarse
 * histogram of segment sizes); a hit returns the stored result without timing,
 * a miss appends the new one.  Synchronizes `stream` (reads seg_off to the
 * host); not to be captured in a graph.  Workspace as kpa_batch_sort with the
 * default configuration.  keys_out/rids_out hold the sorted batch on return
 * unless the cache answered. */
kpa_status kpa_batch_autotune(const uint64_t* keys_in, const uint32_t* rids_in,
                              uint64_t* keys_out, uint32_t* rids_out, const uint64_t* seg_off,
                              uint32_t n_seg, uint64_t n_cap, kpa_sort_algo large_algo,
                              const kpa_pwl_model* models, void* ws, size_t ws_bytes,
                              uint32_t reps, const char* cache_path, kpa_batch_config* best,
                              float* best_ms, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Graph capture of a sequence of calls (launch overhead of a many-launch
 * epoch paid once).  kpa_graph_begin starts capturing `stream` (not the null
 * stream; per-kernel timing must be off); every library call enqueued on it
 * until kpa_graph_end is recorded, not run.  kpa_graph_end instantiates the
 * graph into *out (owned by the caller, freed by kpa_graph_destroy).
 * kpa_graph_launch replays it on `stream`.  The library's launches take their
 * sizes from device memory and record no memsets or host copies, so a replay
 * reads the current contents of the same buffers; host-side arguments (n_cap,
 * n_seg, pointers, configurations) are frozen at capture. */
typedef struct kpa_graph_s* kpa_graph;
kpa_status kpa_graph_begin(hipStream_t stream);
kpa_status kpa_graph_end(hipStream_t stream, kpa_graph* out);
kpa_status kpa_graph_launch(kpa_graph graph, hipStream_t stream);
kpa_status kpa_graph_destroy(kpa_graph graph);

/* ---------------------------------------------------------------------------
 * Merge (Table 2: two sorted KPAs -> one sorted KPA, sequential).  Stable: on
 * equal keys every entry of A precedes every entry of B.  All arrays device;
 * outputs hold na+nb entries and must not alias the inputs.
 */
kpa_status kpa_merge_workspace_size(uint64_t na, uint64_t nb, size_t* bytes);
kpa_status kpa_merge(const uint64_t* a_keys, const uint32_t* a_rids, uint64_t na,
                     const uint64_t* b_keys, const uint32_t* b_rids, uint64_t nb,
                     uint64_t* out_keys, uint32_t* out_rids, void* ws, size_t ws_bytes,
                     hipStream_t stream);
/* Merge n_runs consecutive sorted runs [run_off[r], run_off[r+1]) of one array
 * (run_off: HOST array of n_runs+1 u64) into one sorted KPA of
 * n = run_off[n_runs] - run_off[0] entries at out_keys/out_rids[0, n); ties
 * keep run order.  keys/rids are used as scratch and hold garbage afterwards.
 * Pairwise rounds over the nonempty runs (Sec. 4.2: merges of sorted KPAs at
 * window close); with up to 1024 nonempty runs each round is two launches
 * over all of its pairs and the call makes no host-to-device copy, so it can
 * be captured in a graph (offsets frozen at capture); more runs are merged
 * pair by pair. */
kpa_status kpa_merge_runs_workspace_size(uint64_t n, size_t* bytes);
kpa_status kpa_merge_runs(uint64_t* keys, uint32_t* rids, const uint64_t* run_off,
                          uint32_t n_runs, uint64_t* out_keys, uint32_t* out_rids, void* ws,
                          size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Keyed reduction (Table 2; Sec. 4.2 keyed aggregation: scan a sorted KPA,
 * follow the pointers, coalesce a nonresident column over each run of equal
 * keys).  Input: a KPA sorted by key within each segment (segments as in
 * kpa_sort_segmented); rows: device arena of full records (the rids index it).
 * rids may be NULL: entry i's row is then row i of `rows`, e.g. a value
 * column that kpa_sort_segmented_vals or kpa_batch_sort_vals carried into
 * the KPA's order, read with a layout of 8-byte rows (row_bytes 8, val_off 0,
 * val_w 8).
 * A group is a maximal run of equal keys inside one segment.  For each group,
 * in order: out_gkey = key, out_cnt = entries, out_sum = sum of values mod
 * 2^64, out_max = largest value, out_gstart = index of its first entry.  Any
 * of out_cnt/out_sum/out_max/out_gstart may be NULL.  Outputs (device) need
 * capacity n_cap.  out_gseg_off (device, n_seg+1 u64): first group of each
 * segment and the total number of groups.
 */
kpa_status kpa_reduce_by_key_workspace_size(uint64_t n_cap, uint32_t n_seg, size_t* bytes);
kpa_status kpa_reduce_by_key(const uint64_t* keys, const uint32_t* rids, const uint64_t* seg_off,
                             uint32_t n_seg, uint64_t n_cap, const void* rows,
                             const kpa_row_layout* layout, uint64_t* out_gkey, uint64_t* out_cnt,
                             uint64_t* out_sum, uint64_t* out_max, uint64_t* out_gstart,
                             uint64_t* out_gseg_off, void* ws, size_t ws_bytes,
                             hipStream_t stream);

/* The same keyed reduction for callers that cannot allocate (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): no
 * workspace argument; the reduction's bookkeeping lives in a static 4 MiB
 * device array of the library (one per GPU, held until the process ends), so
 * the call allocates nothing.  It serves n_cap up to about 2^29 entries over a
 * few segments (more: KPA_EUNSUPPORTED, nothing enqueued).  Every call on a
 * GPU uses that GPU's one array: calls that overlap on one GPU (other
 * streams, other threads) race and must be serialized by the caller.
 * Per-kernel timing must be off (KPA_EINVAL otherwise).  Arguments and
 * outputs as kpa_reduce_by_key. */
kpa_status kpa_reduce_by_key_noalloc(const uint64_t* keys, const uint32_t* rids,
                                     const uint64_t* seg_off, uint32_t n_seg, uint64_t n_cap,
                                     const void* rows, const kpa_row_layout* layout,
                                     uint64_t* out_gkey, uint64_t* out_cnt, uint64_t* out_sum,
                                     uint64_t* out_max, uint64_t* out_gstart,
                                     uint64_t* out_gseg_off, hipStream_t stream);

/* Top-k groups per segment by sum: descending sum, ascending key among equal
 * sums (k <= 16).  gkey/gsum/gseg_off as produced by kpa_reduce_by_key.
 * out_key/out_sum: device, n_seg*k entries (segment s at s*k); out_n: device,
 * n_seg u32, the number written (min(k, groups of s)).  g_cap: host upper
 * bound on the total number of groups. */
kpa_status kpa_topk_by_sum_workspace_size(uint64_t g_cap, uint32_t n_seg, size_t* bytes);
kpa_status kpa_topk_by_sum(const uint64_t* gkey, const uint64_t* gsum, const uint64_t* gseg_off,
                           uint32_t n_seg, uint64_t g_cap, uint32_t k, uint64_t* out_key,
                           uint64_t* out_sum, uint32_t* out_n, void* ws, size_t ws_bytes,
                           hipStream_t stream);

/* Median per key (Sec. 6 "Windowed Median Per Key"; percentile by key via sort
 * and reduction, Sec. 4.2): for each group (as in kpa_reduce_by_key) the lower
 * median of its values, v[(c-1)/2] of the ascending values.  Outputs: out_gkey,
 * out_med (device, capacity n_cap), out_gseg_off (device, n_seg+1).  out_cnt
 * and out_sum (device, capacity n_cap each, may be NULL): each group's count
 * and sum of values (mod 2^64), as kpa_reduce_by_key gives them; the values
 * are read once for both the medians and the sums. */
kpa_status kpa_median_by_key_workspace_size(uint64_t n_cap, uint32_t n_seg, size_t* bytes);
kpa_status kpa_median_by_key(const uint64_t* keys, const uint32_t* rids, const uint64_t* seg_off,
                             uint32_t n_seg, uint64_t n_cap, const void* rows,
                             const kpa_row_layout* layout, uint64_t* out_gkey, uint64_t* out_med,
                             uint64_t* out_gseg_off, uint64_t* out_cnt, uint64_t* out_sum,
                             void* ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Join (Table 2: two sorted KPAs, one pass; Sec. 4.2 "Temporal Join").  For
 * each segment s (a window), over all pairs (l, r) of L's segment s and R's
 * segment s with equal keys: out_count[s] = number of pairs, out_sumprod[s] =
 * sum of val(l)*val(r) mod 2^64.  Both KPAs sorted by key within segments;
 * l_seg_off/r_seg_off: device, n_seg+1 each.  rows_l/rows_r: the two arenas
 * (same layout).  out_count/out_sumprod: device, n_seg u64 each.  If out_pairs
 * (device, pairs_cap triples of u64 {key, ridL, ridR}) is not NULL, the pairs
 * are written in (segment, key, ridL, ridR) order up to pairs_cap of them;
 * *out_npairs (device u64, may be NULL) receives the total number of pairs of
 * all segments, so a caller sees that the capacity was too small when
 * *out_npairs > pairs_cap.
 */
kpa_status kpa_join_workspace_size(uint64_t nl_cap, uint64_t nr_cap, uint32_t n_seg,
                                   size_t* bytes);
kpa_status kpa_join(const uint64_t* lk, const uint32_t* lr, const uint64_t* l_seg_off,
                    uint64_t nl_cap, const uint64_t* rk, const uint32_t* rr,
                    const uint64_t* r_seg_off, uint64_t nr_cap, uint32_t n_seg,
                    const void* rows_l, const void* rows_r, const kpa_row_layout* layout,
                    uint64_t* out_count, uint64_t* out_sumprod, uint64_t* out_pairs,
                    uint64_t pairs_cap, uint64_t* out_npairs, void* ws, size_t ws_bytes,
                    hipStream_t stream);

/* Join of two run lists (Table 2 Join; Sec. 4.2 "Temporal Join"), for callers
 * that already hold each side's groups: per segment s, the runs of equal keys
 * of L and of R (key, count, sum of values), keys ascending and unique within
 * a segment of a list, as kpa_reduce_by_key or kpa_median_by_key (with out_cnt
 * and out_sum) write them.  A key present on both sides contributes
 * count_L*count_R pairs and sum_L*sum_R to the sum of value products, so
 * out_count[s] and out_sumprod[s] (device, n_seg u64 each) equal kpa_join's on
 * the KPAs the lists come from.  l_gseg_off/r_gseg_off: device, n_seg+1 each
 * (group offsets per segment); gl_cap/gr_cap: host upper bounds on the groups
 * of each list (< 2^32; too small a bound gives wrong sums, never an access
 * beyond the workspace).  No pairs are written. */
kpa_status kpa_join_runs_workspace_size(uint64_t gl_cap, uint64_t gr_cap, uint32_t n_seg,
                                        size_t* bytes);
kpa_status kpa_join_runs(const uint64_t* l_gkey, const uint64_t* l_cnt, const uint64_t* l_sum,
                         const uint64_t* l_gseg_off, uint64_t gl_cap, const uint64_t* r_gkey,
                         const uint64_t* r_cnt, const uint64_t* r_sum, const uint64_t* r_gseg_off,
                         uint64_t gr_cap, uint32_t n_seg, uint64_t* out_count,
                         uint64_t* out_sumprod, void* ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Materialize (Table 2: KPA -> bundle, random access): out_rows[i] =
 * rows[rids[i]] (row_bytes each).  All device. */
kpa_status kpa_materialize(const uint32_t* rids, uint64_t n, const void* rows, uint32_t row_bytes,
                           void* out_rows, hipStream_t stream);

/* Materialize coalesced with Extract (Sec. 4.3, first optimization: as a
 * primitive emits rows it extracts the KPA the next operator needs): out_rows
 * as kpa_materialize, and from each emitted row the next KPA on the u64
 * column at key_off: out_keys[i] = that column of out_rows row i, out_rids[i]
 * = rid_base + i (pointers into out_rows).  All device; row_bytes a multiple
 * of 8 in [8, 256]; key_off 8-aligned. */
kpa_status kpa_materialize_extract(const uint32_t* rids, uint64_t n, const void* rows,
                                   uint32_t row_bytes, uint32_t key_off, uint32_t rid_base,
                                   void* out_rows, uint64_t* out_keys, uint32_t* out_rids,
                                   hipStream_t stream);

/* ---------------------------------------------------------------------------
 * KeySwap (Table 2: KPA(c1) -> KPA(c2), random access): out_keys[i] = the
 * column of width col_w (4 or 8, zero-extended) at col_off of row rids[i].
 * The rids stay as they are, so (out_keys, rids) is the KPA on the new
 * column.  All device.  out_keys may be the old key array. */
kpa_status kpa_keyswap(const uint32_t* rids, uint64_t n, const void* rows, uint32_t row_bytes,
                       uint32_t col_off, uint32_t col_w, uint64_t* out_keys, hipStream_t stream);

/* In-place update of resident keys (Sec. 4.3, second optimization; the
 * external join of the pipeline example, which replaces each key by the value
 * a small key-value table in device memory holds for it): every keys[i] found
 * among table_keys is replaced by the matching table_vals entry; keys not in
 * the table are left as they are and counted in *out_missing (device u64,
 * set by the call).  table_keys (device, table_n) must be ascending and
 * distinct (otherwise the result is unspecified); tables of up to 2048
 * entries are searched in on-chip memory. */
kpa_status kpa_key_update(uint64_t* keys, uint64_t n, const uint64_t* table_keys,
                          const uint64_t* table_vals, uint64_t table_n, uint64_t* out_missing,
                          hipStream_t stream);

/* Write-back of dirty resident keys (Sec. 4.3, second optimization): the u64
 * column at col_off (8-aligned) of row rids[i] becomes keys[i], so that later
 * KeySwap and Materialize read the updated value.  rows: device, written.
 * Distinct rids write distinct rows; for repeated rids one of the writes
 * wins. */
kpa_status kpa_key_writeback(const uint64_t* keys, const uint32_t* rids, uint64_t n, void* rows,
                             uint32_t row_bytes, uint32_t col_off, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Select (Table 2: KPA -> KPA, keep the pairs that pass; ParDo filters run as
 * Select, Sec. 4.2).  For every segment s (segments as in kpa_sort_segmented)
 * entry i passes when
 *     x_i * den[s]  <op>  num[s]
 * with x_i the resident key (KPA_SEL_KEY) or the value column of its row
 * (KPA_SEL_VALUE, layout->val_off/val_w), the product taken exactly in 128
 * bits and num[s] = num_lo[s] + 2^64 * num_hi[s].  num_hi (NULL: 0) and den
 * (NULL: 1) are optional; with den = 1 and num_hi = 0 this is a plain
 * threshold, and a ratio threshold such as an average sum/count is compared
 * without rounding.  Survivors keep their order and are written back to back
 * (segment after segment) to out_keys/out_rids (device, n_cap each);
 * out_seg_off (device, n_seg+1) receives where each segment's survivors begin
 * and the total.  rows may be NULL for KPA_SEL_KEY. */
typedef enum kpa_select_column { KPA_SEL_KEY = 0, KPA_SEL_VALUE = 1 } kpa_select_column;
typedef enum kpa_select_op {
  KPA_SEL_GT = 0, KPA_SEL_GE = 1, KPA_SEL_LT = 2, KPA_SEL_LE = 3, KPA_SEL_EQ = 4, KPA_SEL_NE = 5
} kpa_select_op;
kpa_status kpa_select_workspace_size(uint64_t n_cap, uint32_t n_seg, size_t* bytes);
kpa_status kpa_select(const uint64_t* keys, const uint32_t* rids, const uint64_t* seg_off,
                      uint32_t n_seg, uint64_t n_cap, const void* rows,
                      const kpa_row_layout* layout, kpa_select_column column, kpa_select_op op,
                      const uint64_t* num_lo, const uint64_t* num_hi, const uint64_t* den,
                      uint64_t* out_keys, uint32_t* out_rids, uint64_t* out_seg_off, void* ws,
                      size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Unkeyed reduction over windows (Table 2 "Unkeyed reduction"; Sec. 6
 * "Windowed Average All"): one pass over the rows; for each window w (window
 * rule as kpa_partition_windows) out_cnt[w] = rows in the window,
 * out_sum_lo[w] + 2^64 * out_sum_hi[w] = the exact sum of their values (a
 * 128-bit integer, so the average sum/count can be taken without overflow),
 * out_max[w] = the largest value; *out_oob = rows outside all windows.  Any
 * output may be NULL.  1 <= n_win <= 256, n < 2^32.  All device. */
kpa_status kpa_reduce_all_windows_workspace_size(uint32_t n_win, size_t* bytes);
kpa_status kpa_reduce_all_windows(const void* rows, uint64_t n, const kpa_row_layout* layout,
                                  uint64_t win_len, uint64_t win_origin, uint32_t n_win,
                                  uint64_t* out_cnt, uint64_t* out_sum_lo, uint64_t* out_sum_hi,
                                  uint64_t* out_max, uint64_t* out_oob, void* ws, size_t ws_bytes,
                                  hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Per-key order statistics of the values (Sec. 6 benchmarks "TopK Per Key"
 * and "Unique Count Per Key"), on a KPA sorted by key within segments, rows
 * reached through the rids.  Groups as in kpa_reduce_by_key (out_gkey,
 * out_gseg_off: device, capacity n_cap and n_seg+1).
 * kpa_topk_per_key: per group g, out_gcnt[g] = its entries, out_gstart[g] =
 * the index of its first entry, and its min(k, count) largest values in
 * descending order at out_topv[out_gstart[g] + j], j < min(k, count) (equal
 * values repeat; out_topv: device, n_cap u64, other slots untouched).
 * 1 <= k <= 16.
 * kpa_unique_count_by_key: out_uniq[g] = the number of distinct values of the
 * group.
 * Runs longer than 4096 entries are sorted by value through the radix sort's
 * passes (a run of 2^30 or more entries is not supported). */
kpa_status kpa_run_stats_workspace_size(uint64_t n_cap, uint32_t n_seg, size_t* bytes);
kpa_status kpa_topk_per_key(const uint64_t* keys, const uint32_t* rids, const uint64_t* seg_off,
                            uint32_t n_seg, uint64_t n_cap, const void* rows,
                            const kpa_row_layout* layout, uint32_t k, uint64_t* out_gkey,
                            uint64_t* out_gcnt, uint64_t* out_gstart, uint64_t* out_topv,
                            uint64_t* out_gseg_off, void* ws, size_t ws_bytes,
                            hipStream_t stream);
kpa_status kpa_unique_count_by_key(const uint64_t* keys, const uint32_t* rids,
                                   const uint64_t* seg_off, uint32_t n_seg, uint64_t n_cap,
                                   const void* rows, const kpa_row_layout* layout,
                                   uint64_t* out_gkey, uint64_t* out_uniq, uint64_t* out_gseg_off,
                                   void* ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Sliding windows (Sec. 4.2 "Windowing": a sliding window is built from
 * partitions whose range is the slide length).  With the rows partitioned into
 * panes of one slide each, sorted and reduced per pane (gkey, gseg_off as
 * produced by kpa_reduce_by_key over n_pane segments), window w of length
 * panes_per_window slides covers panes w .. w+panes_per_window-1;
 * n_win = n_pane - panes_per_window + 1 <= 65535.  Writes, window after
 * window, the concatenation of those panes' groups as a KPA of (group key,
 * group index): out_keys/out_rids (device, out_cap), out_seg_off (device,
 * n_win+1; the last entry is the total, possibly above out_cap, in which case
 * only the first out_cap entries are written).  Sorting each window's
 * segment and reducing it with the pane groups' count, sum and max columns as
 * values gives the sliding window's aggregates. */
kpa_status kpa_window_panes(const uint64_t* gkey, const uint64_t* gseg_off, uint32_t n_pane,
                            uint32_t panes_per_window, uint64_t* out_keys, uint32_t* out_rids,
                            uint64_t* out_seg_off, uint64_t out_cap, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * The two alternatives the paper measures its KPA grouping against.
 *
 * Grouping on full rows (the design without KPAs of the ablation in Sec. 7.3):
 * out_rows receives all n rows ordered by (window, key), stably, so each
 * window's rows are grouped by key in arrival order; rows in no window (window
 * rule as kpa_partition_windows) count as window n_win and come last.
 * out_win_off (device, n_win+1) delimits the windows; *out_oob (device) counts
 * the rows after out_win_off[n_win].  Nine onesweep passes move whole rows (the
 * eight key bytes, then the window).  row_bytes 16 or 32, n < 2^30,
 * 1 <= n_win <= 255; rows and out_rows device, not aliased. */
kpa_status kpa_sort_rows_windowed_workspace_size(uint64_t n, uint32_t row_bytes, size_t* bytes);
kpa_status kpa_sort_rows_windowed(const void* rows, uint64_t n, const kpa_row_layout* layout,
                                  uint64_t win_len, uint64_t win_origin, uint32_t n_win,
                                  void* out_rows, uint64_t* out_win_off, uint64_t* out_oob,
                                  void* ws, size_t ws_bytes, hipStream_t stream);

/* Hash GroupBy (Sec. 2.2: the random-access alternative, an open-addressing
 * pre-allocated table): per distinct key of the rows, count, sum (mod 2^64)
 * and max of the value column, in the table's order (not sorted by key).
 * table_cap: slots, a power of two up to 2^31, larger than the number of
 * distinct keys (linear probing).  Up to g_cap groups are written to
 * out_gkey/out_cnt/out_sum/out_max (device; the last three may be NULL);
 * *out_ngroups (device) receives the number of groups, or all ones when a key
 * found no free slot (table_cap too small).  All device. */
kpa_status kpa_hash_groupby_workspace_size(uint64_t table_cap, size_t* bytes);
kpa_status kpa_hash_groupby(const void* rows, uint64_t n, const kpa_row_layout* layout,
                            uint64_t table_cap, uint64_t* out_gkey, uint64_t* out_cnt,
                            uint64_t* out_sum, uint64_t* out_max, uint64_t g_cap,
                            uint64_t* out_ngroups, void* ws, size_t ws_bytes,
                            hipStream_t stream);

/* ---------------------------------------------------------------------------
 * CDF models for the learned-splitter sort.
 *
 * kpa_pwl_fit: for each segment of a sorted KPA, kmin/kmax = first/last key and
 * knots[j] = (number of keys < kmin + floor(j*(kmax-kmin)/n_seg_model)) / n,
 * rounded once to float.  Empty segments get n_seg = 0.  out_models: device,
 * n_seg entries.
 */
kpa_status kpa_pwl_fit(const uint64_t* sorted_keys, const uint64_t* seg_off, uint32_t n_seg,
                       uint32_t n_seg_model, kpa_pwl_model* out_models, hipStream_t stream);

/* Monotone CDF network 1 -> 32 -> 32 -> 1 (nonnegative weights, ramp
 * activation r(z) = min(max(z,0),1)); parameters as 1153 floats
 * [W1(32), b1(32), W2(32x32 row-major, W2[o][i]), b2(32), W3(32), b3].
 * kpa_mlp_training_set: S training pairs from a sorted KPA of n keys: sample
 * s takes index i = floor(s*n/S); x = (key_i - kmin)/(kmax - kmin) in float
 * (0 when kmax == kmin), y = i/n.  Writes x, y (device, S floats) and the
 * model range into out_model->kmin/kmax. */
#define KPA_MLP_PARAMS 1153
kpa_status kpa_mlp_training_set(const uint64_t* sorted_keys, uint64_t n, uint32_t S, float* x,
                                float* y, kpa_pwl_model* out_model, hipStream_t stream);
kpa_status kpa_mlp_forward(const float* params, const float* x, uint32_t m, float* out_f,
                           hipStream_t stream);
/* Mean squared error and its gradient over m samples (deterministic). */
kpa_status kpa_mlp_loss_grad_workspace_size(uint32_t m, size_t* bytes);
kpa_status kpa_mlp_loss_grad(const float* params, const float* x, const float* y, uint32_t m,
                             float* out_loss, float* out_grad, void* ws, size_t ws_bytes,
                             hipStream_t stream);
/* One Adam step (step number t >= 1), then weights projected onto >= 0. */
kpa_status kpa_mlp_adam_step(float* params, const float* grad, float* adam_m, float* adam_v,
                             uint32_t t, float lr, float beta1, float beta2, float eps,
                             hipStream_t stream);
/* `steps` full-batch Adam steps starting at step t0 (loss of the last step in
 * *out_loss, device float, may be NULL). */
kpa_status kpa_mlp_train(float* params, float* adam_m, float* adam_v, const float* x,
                         const float* y, uint32_t m, uint32_t t0, uint32_t steps, float lr,
                         float* out_loss, void* ws, size_t ws_bytes, hipStream_t stream);
/* Starting parameters from 1153 caller-supplied uniforms in [0, 1) (device;
 * the network's random initialization drawn by the caller): W1 = 4 + 4u
 * (slopes in [4, 8)), b1 = -W1 * (i + u')/32 (breakpoints spread over [0, 1]),
 * W2 = (0.5 + u)/32, b2 = -0.25 + 0.5u, W3 = (0.5 + u)/32, b3 = 0; u, u'
 * the uniform at the parameter's own index, u' the one at index 32 + i. */
kpa_status kpa_mlp_init(const float* uniforms, float* params, hipStream_t stream);
/* Distill the network into model->knots: F_j = running max of clamp(f(j/n_seg),
 * 0, 1), j = 0..n_seg; kmin/kmax are kept from kpa_mlp_training_set. */
kpa_status kpa_mlp_to_pwl(const float* params, uint32_t n_seg_model, kpa_pwl_model* model,
                          hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Ingest (the engine receives record bundles in arrival order and keeps them
 * as rows; Sec. 3 and 5): copies n rows from host memory (pinned for an
 * asynchronous copy) to dev_rows (device, n*row_bytes, 16-byte aligned) on
 * `stream` and, when ts_add != 0, adds ts_add (mod 2^64 for 8-byte, mod 2^32
 * for 4-byte timestamps) to every row's timestamp on the device, so that a
 * replayed bundle can be moved to a new event time.  The caller assigns rids
 * (e.g. rid_base of kpa_partition_windows = the rows' arena index). */
kpa_status kpa_ingest_bundle(const void* host_rows, uint64_t n, const kpa_row_layout* layout,
                             uint64_t ts_add, void* dev_rows, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Serving loop (the runtime of Sec. 3 and 5: bundles processed as they
 * arrive, windows closed by watermarks, merge of the window's sorted runs at
 * close, a reserved pool for that urgent work, back-pressure when memory is
 * short).  A server owns one device allocation of budget_bytes, `slots`
 * streams for bundle work and one for window closes (all at the default
 * priority), a dispatcher and a closer thread.
 *
 * Queries: KPA_Q_SUM (per key count/sum/max, top-10 keys by sum),
 * KPA_Q_MEDIAN (lower median per key), KPA_Q_JOIN (two sides; per window the
 * number of equal-key pairs and the sum of value products mod 2^64).  Windows
 * are tumbling: [origin + w*win_len, origin + (w+1)*win_len).
 *
 * kpa_server_submit: one bundle of n rows (host memory that must stay valid
 * and unchanged until kpa_server_drain returns or the server is destroyed;
 * pinned memory for asynchronous copies) for query qid, side 0 (or 1 for the
 * right side of a join).  Row timestamps are taken as ts + ts_base; every row
 * must satisfy ts_lo <= ts <= ts_hi (the producer's bounds), and the bundle
 * may span at most 8 windows.  The bundle is queued; the dispatcher admits it
 * when a slot, ring rows and pool memory are free (rows of windows already
 * closed are dropped and counted as late).  When max_pending bundles are
 * queued, a blocking submit waits and a non-blocking one returns
 * KPA_EBUDGET (back-pressure).
 * kpa_server_watermark: no row with timestamp < t will follow for qid; every
 * window of qid ending at or before t that received rows is closed and
 * yields one kpa_window_result.  Watermarks are queued in order with the
 * bundles and never refused.
 * kpa_server_poll: takes one finished result (waits up to timeout_ms; *got=0
 * if none).  kpa_server_drain: waits until every queued bundle and watermark
 * has been processed and every close has finished (timeout_ms < 0: no limit;
 * KPA_ETIMEOUT when the limit passes first, the server running on).
 * Latency of a window = time its result reached the host - time the closing
 * watermark was submitted.
 * A failure inside the server threads stops it; later calls return the
 * failing status with the message in kpa_last_error_string().  Only window
 * closes free pool memory, so nothing waits for memory that no close would
 * free: a window close that needs more device memory than is free (the
 * close reserve and unused pool) stops the server with KPA_EBUDGET; and when
 * a bundle finds no memory or record while no close is queued or running,
 * the server is stalled until a watermark closes a window: a blocking submit
 * that finds the queue full then returns KPA_EBUDGET instead of waiting, and
 * so does drain (the server runs on and a later watermark resumes it). */
typedef enum kpa_query_kind { KPA_Q_SUM = 0, KPA_Q_MEDIAN = 1, KPA_Q_JOIN = 2 } kpa_query_kind;

typedef struct kpa_server_config {
  uint64_t budget_bytes;     /* device memory of the server, allocated once */
  uint32_t slots;            /* bundles on the device at once (1..64) */
  uint32_t rows_in_host;     /* 1: full rows are not kept in device memory */
  uint64_t max_bundle_rows;  /* largest bundle */
  uint32_t max_row_bytes;    /* largest row of any query (multiple of 8, <= 256) */
  uint32_t max_pending;      /* queued bundles before submit applies back-pressure */
  uint32_t reserve_pct;      /* % of the pool reserved for window closes (<= 90) */
  uint32_t max_live_bundles; /* bundles admitted and not yet released */
  /* Capacity tier (Sec. 5): pinned host memory that holds bundle KPAs (sorted
   * keys and values) the placement sends there; kernels of the window close
   * read them over the host link. */
  uint64_t host_pool_bytes;  /* 0: no capacity tier */
  uint32_t placement;        /* a kpa_placement */
  uint32_t monitor_ms;       /* knob refresh interval (Sec. 5 samples every 10 ms) */
  double target_delay_ms;    /* output delay target of the k_high rule */
  double host_bw_gbs;        /* host-link bandwidth taken as full use (0: measured) */
  uint32_t keep_groups;      /* 1: SUM and MEDIAN results carry their per-key arrays */
  uint32_t seed;             /* seed of the placement draws */
} kpa_server_config;

/* Where new bundle KPAs go.  DEVICE: the device pool (HBM) only.  BALANCED:
 * the paper's policy (Sec. 5): each bundle gets an impact tag from the window
 * it feeds (High: one of the two next windows of its query to close; Low:
 * later) and is placed in HBM with probability k_high or k_low (the demand
 * balance knob), else in the host pool; window-close work (Urgent) always
 * uses the reserved part of the device pool; when the device pool is full a
 * bundle spills to the host pool whatever its tag.  HOST: every bundle KPA in
 * the host pool. */
typedef enum kpa_placement {
  KPA_PLACE_DEVICE = 0, KPA_PLACE_BALANCED = 1, KPA_PLACE_HOST = 2
} kpa_placement;

/* One refresh of the demand balance knob (Sec. 5), as the server's monitor
 * applies it every monitor_ms.  hbm_util: fraction of the device pool
 * outside the close reserve that bundles hold; bw_util: host-link use (rows
 * in at ingest, host-pool KPAs out and back) over what the link carries at
 * host_bw_gbs, smoothed over about 100 ms.  When capacity is the tighter resource (hbm_util exceeds
 * bw_util by more than 0.1) new KPAs move toward the host (step -0.05), when
 * bandwidth is, toward HBM (+0.05), else nothing changes.  The step goes to
 * k_low unless k_low already sits at the end it moves toward; then to k_high,
 * but only when the current output delay is at least 10% below the target
 * (delay_ms <= 0.9 * target_ms).  Both stay in [0, 1]; they start at 1. */
kpa_status kpa_balance_knob_update(double* k_low, double* k_high, double hbm_util,
                                   double bw_util, double delay_ms, double target_ms);

typedef struct kpa_window_result {
  uint32_t query;
  uint32_t kind;        /* kpa_query_kind */
  uint64_t window;      /* w: [origin + w*win_len, origin + (w+1)*win_len) */
  uint64_t rows[2];     /* entries of the window per side */
  uint64_t groups;      /* SUM/MEDIAN: distinct keys; JOIN: number of pairs */
  uint64_t total;       /* SUM: sum of all values; JOIN: sum of value products (mod 2^64) */
  uint64_t digest;      /* SUM/MEDIAN: sum over keys of h (mod 2^64), see below */
  uint32_t n_top;       /* SUM: number of top keys (<= 10) */
  uint32_t reserved;
  uint64_t top_key[10]; /* SUM: keys by descending sum, ascending key */
  uint64_t top_sum[10];
  double latency_ms;
  /* keep_groups: the window's per-key arrays in host memory owned by the
   * server until kpa_server_release_groups(groups_data): SUM: gkey[G], cnt[G],
   * sum[G], max[G]; MEDIAN: gkey[G], median[G] (G = groups, ascending key).
   * NULL otherwise (and for JOIN). groups_words = u64 words at groups_data. */
  const uint64_t* groups_data;
  uint64_t groups_words;
  uint32_t runs;        /* bundle runs merged for the window (all sides) */
  uint32_t runs_host;   /* of which read from the host pool */
} kpa_window_result;
/* digest: with m(z) the SplitMix64 finalizer (z ^= z>>30; z *= 0xBF58476D1CE4E5B9;
 * z ^= z>>27; z *= 0x94D049BB133111EB; z ^= z>>31), SUM: h = m(key ^ m(count ^
 * m(sum ^ m(max)))); MEDIAN: h = m(key ^ m(median ^ m(0 ^ m(0)))).  It depends
 * on every per-key result but not on their order. */

typedef struct kpa_server_stats {
  uint64_t bundles;            /* admitted */
  uint64_t rows;               /* admitted rows */
  uint64_t late_rows;          /* rows outside the open windows (dropped) */
  uint64_t windows_closed;
  uint64_t backpressure_waits; /* admissions that had to wait */
  uint64_t pool_peak_bytes;
  uint64_t pool_bytes;
  double p50_ms, p99_ms, max_ms; /* window latency */
  double elapsed_s;            /* first submit -> last result */
  double mrec_per_s;           /* admitted rows / elapsed_s */
  uint64_t bundles_on_host;    /* bundle KPAs placed in the host pool */
  uint64_t host_pool_bytes;    /* host pool in use now */
  uint64_t host_pool_peak_bytes;
  double k_low, k_high;        /* current demand balance knob */
  double host_bw_gbs;          /* host-link bandwidth taken as full use */
} kpa_server_statistics;

/* One sample of the server's monitor (every monitor_ms). */
typedef struct kpa_monitor_sample {
  double t_s;            /* since the first submit */
  double hbm_util;       /* device pool held by bundles / the pool outside the close reserve */
  double bw_util;        /* host-link use: bytes moved (rows in at ingest, host-pool KPAs
                            out and back) / what the link carries, smoothed over ~100 ms */
  double k_low, k_high;
  double delay_ms;       /* current output delay: largest latency of the last 16 windows */
  uint64_t hbm_bytes;    /* device pool in use */
  uint64_t host_bytes;   /* host pool in use */
  uint64_t waits;        /* admissions that had to wait so far (back-pressure) */
  uint64_t bundles_host; /* bundle KPAs placed in the host pool so far */
} kpa_monitor_sample;

typedef struct kpa_server_s* kpa_server;

/* budget 64 GiB, 8 slots, rows in device memory, bundles up to 2^20 rows of
 * up to 32 bytes, 256 pending, 25% reserve, 65536 live bundles, no host pool,
 * device placement, 10 ms monitor, 1000 ms target delay, host-link bandwidth
 * measured, no per-key arrays, seed 1.  A bundle needs 16 bytes per row in a
 * pool (plus its rows in the device pool unless rows_in_host); creation fails
 * with KPA_EBUDGET when the largest bundle could never be admitted. */
kpa_status kpa_server_config_default(kpa_server_config* cfg);
kpa_status kpa_server_create(const kpa_server_config* cfg, kpa_server* out);
/* A bundle's memory (sorted keys and values, plus the rows when they are kept
 * on the device) is taken from the pool at admission and returned when every
 * window it has rows in is closed. */
kpa_status kpa_server_add_query(kpa_server server, kpa_query_kind kind,
                                const kpa_row_layout* layout, uint64_t win_len,
                                uint64_t win_origin, uint32_t* qid);
kpa_status kpa_server_submit(kpa_server server, uint32_t qid, uint32_t side, const void* rows,
                             uint64_t n, uint64_t ts_base, uint64_t ts_lo, uint64_t ts_hi,
                             int32_t blocking);
kpa_status kpa_server_watermark(kpa_server server, uint32_t qid, uint64_t t);
kpa_status kpa_server_poll(kpa_server server, kpa_window_result* out, int32_t* got,
                           int32_t timeout_ms);
kpa_status kpa_server_drain(kpa_server server, int32_t timeout_ms);
kpa_status kpa_server_stats(kpa_server server, kpa_server_statistics* out);
/* Frees the per-key arrays of a result (keep_groups). */
kpa_status kpa_server_release_groups(kpa_server server, const uint64_t* groups_data);
/* Copies up to cap monitor samples (the oldest first) and sets *n to the
 * number copied; the server keeps the latest 65536. */
kpa_status kpa_server_trace(kpa_server server, kpa_monitor_sample* out, uint32_t cap,
                            uint32_t* n);
kpa_status kpa_server_destroy(kpa_server server);

#ifdef __cplusplus
}
#endif
#endif /* KPA_H_ */
