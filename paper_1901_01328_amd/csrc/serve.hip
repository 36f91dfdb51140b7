// Serving loop: record bundles arrive as they are produced, are admitted onto
// the GPU as slots and memory allow, and window results come back when a
// watermark closes the window.  This is the runtime side of the paper's
// engine (Sec. 3 and 5): bundles processed as they come (data parallelism
// over bundles), watermarks as the signal that a window is complete, window
// close = merge of the window's sorted runs then the keyed operator, a
// reserved memory pool for the urgent close work, and back-pressure on the
// producer when memory runs out.
//
// Per bundle (dispatcher thread, on one of `slots` streams): ingest
// (host -> device copy, timestamps rebased), partition into the windows the
// bundle touches with the value column staged, stable sort of each window's
// part, and the values gathered into the sorted order.  The bundle keeps its
// sorted runs (key and value per entry) in the pool until every window it
// touches is closed, then releases them; nothing is held in arrival order, so
// a bundle that straddles two windows pins only its own memory.
// Per closed window (closer thread, own stream): the runs of all bundles of
// that window are concatenated (keys, and values that the KPA's pointers
// index) and merged into one sorted KPA, then reduced
// (SUM: count/sum/max per key and top-10 by sum; MEDIAN: lower median per
// key; JOIN: merge-join of the two sides' KPAs), and a small summary is
// copied to the host.
//
// Memory: one device allocation of budget_bytes, handed out by an extent
// allocator; reserve_pct of it only serves window-close work, so closes can
// always proceed and free the bundles that hold memory.  All streams run at
// the default priority.
//
// Hybrid placement (Sec. 5): an optional pinned host pool is the capacity
// tier.  Each bundle's KPA (sorted keys and values) goes to the device pool
// or the host pool by its impact tag and the demand balance knob {k_low,
// k_high}; a monitor thread samples device-pool use and host-link traffic
// every monitor_ms and moves the knob.  A KPA placed on the host is sorted in
// the slot's device scratch and copied out; the window close copies it back
// over the host link when it merges the window's runs.
#include "kpa_internal.hpp"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <thread>
#include <vector>

namespace kpa {
namespace {

using Clock = std::chrono::steady_clock;

constexpr u32 MAX_BUNDLE_WINDOWS = 8;
constexpr u64 ALIGN = 256;

// ------------------------------------------------------------- kernels --

// Adds `add` (mod 2^64) to the timestamp of each row (ingest rebase).
__global__ void __launch_bounds__(BLOCK) k_add_ts(unsigned char* __restrict__ rows, u64 n,
                                                  u32 row_bytes, u32 ts_off, u32 ts_w, u64 add) {
  for (u64 i = (u64)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (u64)gridDim.x * BLOCK) {
    unsigned char* p = rows + i * row_bytes + ts_off;
    if (ts_w == 8)
      *reinterpret_cast<u64*>(p) += add;
    else
      *reinterpret_cast<u32*>(p) += (u32)add;
  }
}

__global__ void k_set2(u64* p, u64 a, u64 b) {
  p[0] = a;
  p[1] = b;
}

__device__ __forceinline__ u64 fmix(u64 z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Order-independent fingerprint of a window's per-key results, summed mod
// 2^64 over the groups g < *n_groups:  h = fmix(key ^ fmix(a ^ fmix(b ^
// fmix(c)))) with absent columns taken as 0.  out[1] += sum of b (the SUM
// total).  out must be zeroed first.
__global__ void __launch_bounds__(BLOCK) k_digest(const u64* __restrict__ key,
                                                  const u64* __restrict__ a,
                                                  const u64* __restrict__ b,
                                                  const u64* __restrict__ c,
                                                  const u64* __restrict__ n_groups,
                                                  u64* __restrict__ out) {
  const u64 g = *n_groups;
  u64 h = 0, tb = 0;
  for (u64 i = (u64)blockIdx.x * BLOCK + threadIdx.x; i < g; i += (u64)gridDim.x * BLOCK) {
    const u64 va = a ? a[i] : 0, vb = b ? b[i] : 0, vc = c ? c[i] : 0;
    h += fmix(key[i] ^ fmix(va ^ fmix(vb ^ fmix(vc))));
    tb += vb;
  }
  h = wave_sum(h);
  tb = wave_sum(tb);
  if (__lane_id() == 0) {
    atomicAdd(reinterpret_cast<unsigned long long*>(out), (unsigned long long)h);
    atomicAdd(reinterpret_cast<unsigned long long*>(out + 1), (unsigned long long)tb);
  }
}

// ---------------------------------------------------------------- pool --

// Extents of one device allocation, first fit, 256-byte granules.  Normal
// requests leave `reserve` bytes free; urgent ones may use everything.
class Pool {
 public:
  void init(char* base, u64 size, u64 reserve) {
    base_ = base;
    size_ = size;
    reserve_ = reserve;
    free_.clear();
    free_[0] = size;
    free_bytes_ = size;
  }
  // Returns nullptr when it does not fit now.  Caller holds the server lock.
  void* try_alloc(u64 bytes, bool urgent) {
    bytes = (bytes + ALIGN - 1) / ALIGN * ALIGN;
    if (bytes == 0) bytes = ALIGN;
    if (!urgent && free_bytes_ < bytes + reserve_) return nullptr;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const u64 off = it->first, len = it->second;
        free_.erase(it);
        if (len > bytes) free_[off + bytes] = len - bytes;
        free_bytes_ -= bytes;
        used_peak_ = std::max(used_peak_, size_ - free_bytes_);
        return base_ + off;
      }
    }
    return nullptr;
  }
  void release(void* p, u64 bytes) {
    if (!p) return;
    bytes = (bytes + ALIGN - 1) / ALIGN * ALIGN;
    if (bytes == 0) bytes = ALIGN;
    u64 off = (u64)(static_cast<char*>(p) - base_);
    free_bytes_ += bytes;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && next->first == off + bytes) {
      bytes += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += bytes;
        return;
      }
    }
    free_[off] = bytes;
  }
  bool fits_ever(u64 bytes, bool urgent) const {
    bytes = (bytes + ALIGN - 1) / ALIGN * ALIGN;
    return bytes + (urgent ? 0 : reserve_) <= size_;
  }
  u64 used() const { return size_ - free_bytes_; }
  u64 peak() const { return used_peak_; }
  u64 size() const { return size_; }
  bool owns(const void* p) const {
    const char* c = static_cast<const char*>(p);
    return base_ && c >= base_ && c < base_ + size_;
  }

 private:
  char* base_ = nullptr;
  u64 size_ = 0, reserve_ = 0, free_bytes_ = 0, used_peak_ = 0;
  std::map<u64, u64> free_;
};

// --------------------------------------------------------------- state --

struct Bundle {
  u32 q = 0, side = 0;
  u64 n = 0;
  u64 w_lo = 0;      // first window
  u32 n_win = 0;
  void* block = nullptr;   // the KPA: keys | values, in the device or the host pool
  u64 bytes = 0;
  bool on_host = false;    // the KPA is in the host pool
  void* rblock = nullptr;  // device pool: the rows, when they are kept on the device
  u64 rbytes = 0;
  u64* keys = nullptr;    // sorted runs of the windows, back to back
  u64* vals = nullptr;    // value of each sorted entry
  unsigned char* rows = nullptr;
  u64* h_off = nullptr;   // pinned: window offsets [n_win + 1], then out-of-range count
  hipEvent_t done = nullptr;
  int refs = 0;           // windows of this bundle not yet closed
};

struct Query {
  u32 kind = 0;
  kpa_row_layout layout{};
  u64 win_len = 1, origin = 0;
  int sides = 1;
  u64 next_close = 0;  // first window not closed
  u64 wm = 0;
  bool have_wm = false;
  std::map<u64, std::vector<Bundle*>> by_win[2];
};

struct Cmd {
  enum Kind { BUNDLE, WATERMARK } kind;
  u32 q = 0, side = 0;
  const void* rows = nullptr;
  u64 n = 0, ts_base = 0, ts_lo = 0, ts_hi = 0;
  u64 t = 0;
  Clock::time_point at;
};

struct CloseJob {
  u32 q;
  u64 w;
  Clock::time_point t_ingest;
  std::vector<Bundle*> runs[2];
};

struct Slot {
  hipStream_t st = nullptr;
  hipEvent_t last = nullptr;  // completion of the slot's latest bundle
  bool used = false;
  u64* pkeys = nullptr;  // partition output (max_n)
  u32* prids = nullptr;
  u64* pvals = nullptr;  // staged values in arrival order (max_n)
  u32* srids = nullptr;  // sorted rids (max_n)
  u64* win_off = nullptr;  // MAX_BUNDLE_WINDOWS + 1
  u64* oob = nullptr;
  void* part_ws = nullptr;
  size_t part_ws_bytes = 0;
  void* sort_ws = nullptr;
  size_t sort_ws_bytes = 0;
  unsigned char* staging = nullptr;  // rows when they stay on the host
  u64* okeys = nullptr;  // sorted keys and values of a KPA placed on the host (max_n)
  u64* ovals = nullptr;
};

}  // namespace
}  // namespace kpa

struct kpa_server_s {
  kpa_server_config cfg{};
  int device = 0;
  char* mem = nullptr;
  kpa::Pool pool;
  std::vector<kpa::Slot> slots;
  hipStream_t close_st = nullptr;
  std::vector<std::unique_ptr<kpa::Query>> queries;
  u64* h_records = nullptr;  // pinned per-bundle offset records
  std::vector<u32> free_records;
  std::set<kpa::Bundle*> live_bundles;
  std::vector<hipEvent_t> event_pool;

  std::mutex mu;
  std::condition_variable cv_cmd, cv_space, cv_done, cv_close;
  std::deque<kpa::Cmd> cmds;
  std::deque<kpa::CloseJob> closes;
  std::deque<kpa_window_result> results;
  u64 cmds_in = 0, cmds_done = 0, closes_in = 0, closes_done = 0;
  bool stop = false;
  bool stalled = false;  // the dispatcher waits for memory that no queued close frees
  kpa_status failed = KPA_OK;
  std::string fail_msg;

  // statistics
  u64 n_bundles = 0, n_rows = 0, n_late = 0, n_waits = 0;
  std::vector<double> lat_ms;
  bool started = false;
  kpa::Clock::time_point t_first, t_last;

  // capacity tier and placement
  char* hmem = nullptr;     // pinned host pool
  kpa::Pool hpool;
  double k_low = 1.0, k_high = 1.0;
  u64 rng = 0;              // SplitMix64 counter of the placement draws
  u64 n_host = 0;           // bundle KPAs placed on the host
  u64 host_moved = 0;       // host-link bytes of host-pool KPAs (both directions)
  u64 rows_moved = 0;       // host-link bytes of rows copied in at ingest
  u64 close_bytes = 0;      // device pool held by window closes now (urgent work)
  double host_bw = 0.0;     // GB/s taken as full use of the host link
  std::vector<kpa_monitor_sample> trace;
  std::set<const uint64_t*> groups_out;  // per-key arrays handed to the caller

  std::thread dispatcher, closer, monitor;
};

namespace kpa {
namespace {

using Server = kpa_server_s;

constexpr u32 RECORD_WORDS = MAX_BUNDLE_WINDOWS + 2;

// Stops the server with the first failure.  Caller holds the lock.
void fail_locked(Server* s, kpa_status code, const char* what) {
  if (s->failed == KPA_OK) {
    s->failed = code;
    s->fail_msg = what;
    if (code == KPA_EHIP) {
      s->fail_msg += ": ";
      s->fail_msg += kpa_last_error_string();
    }
  }
  s->stop = true;
  s->cv_cmd.notify_all();
  s->cv_space.notify_all();
  s->cv_done.notify_all();
  s->cv_close.notify_all();
}

void fail(Server* s, kpa_status code, const char* what) {
  std::lock_guard<std::mutex> lk(s->mu);
  fail_locked(s, code, what);
}

// Placement draw of one bundle KPA (Sec. 5): true for the host pool.  High
// bundles stay in HBM with probability k_high, Low ones with k_low.  Caller
// holds the lock.
bool place_on_host(Server* s, bool high) {
  if (!s->hmem || s->cfg.placement == KPA_PLACE_DEVICE) return false;
  if (s->cfg.placement == KPA_PLACE_HOST) return true;
  s->rng += 0x9E3779B97F4A7C15ull;
  u64 z = s->rng;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
  return !(u < (high ? s->k_high : s->k_low));
}

hipEvent_t take_event(Server* s) {
  if (!s->event_pool.empty()) {
    hipEvent_t e = s->event_pool.back();
    s->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  return e;
}

u64 rnd(u64 x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

// Releases a bundle once no window needs it.  Caller holds the lock.
void release_bundle(Server* s, Bundle* b) {
  if (b->on_host) s->hpool.release(b->block, b->bytes);
  else s->pool.release(b->block, b->bytes);
  if (b->rblock) s->pool.release(b->rblock, b->rbytes);
  s->free_records.push_back((u32)((b->h_off - s->h_records) / RECORD_WORDS));
  if (b->done) s->event_pool.push_back(b->done);
  s->live_bundles.erase(b);
  delete b;
}

// vals_out[i] = vals[rids[i]] for i < *count (values into sorted order).
__global__ void __launch_bounds__(BLOCK) k_gather_vals(const u32* __restrict__ rids,
                                                       const u64* __restrict__ vals,
                                                       const u64* __restrict__ count,
                                                       u64* __restrict__ out) {
  const u64 n = *count;
  for (u64 i = (u64)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (u64)gridDim.x * BLOCK)
    out[i] = vals[rids[i]];
}

__global__ void __launch_bounds__(BLOCK) k_iota(u32* __restrict__ out, u64 n) {
  for (u64 i = (u64)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (u64)gridDim.x * BLOCK)
    out[i] = (u32)i;
}

// --------------------------------------------------------- dispatcher --

void close_windows(Server* s, const Cmd& c);

// While bundle B waits for memory or a slot, watermarks queued behind it
// may be the only way to free them.  A queued watermark is applied early
// when it cannot close a window that a bundle still waiting before it (B
// included) has rows in.  Caller holds the lock.
void early_watermarks(Server* s, u32 qb, u64 wb_lo) {
  std::vector<std::pair<u32, u64>> waiting{{qb, wb_lo}};  // (query, first window) of bundles ahead
  for (auto it = s->cmds.begin(); it != s->cmds.end();) {
    if (it->kind == Cmd::BUNDLE) {
      const Query& q = *s->queries[it->q];
      const u64 lo_t = it->ts_base + it->ts_lo;
      waiting.push_back({it->q, lo_t >= q.origin ? (lo_t - q.origin) / q.win_len : 0});
      ++it;
      continue;
    }
    const Query& q = *s->queries[it->q];
    const u64 closable = it->t >= q.origin ? (it->t - q.origin) / q.win_len : 0;
    bool safe = true;
    for (auto& wq : waiting)
      if (wq.first == it->q && closable > wq.second) safe = false;
    if (safe) {
      close_windows(s, *it);
      it = s->cmds.erase(it);
      s->cmds_in--;  // applied here, outside the dispatcher's count
      s->cv_space.notify_all();
    } else {
      ++it;
    }
  }
}

// Admits and launches one bundle.  Returns false when the server stops.
bool run_bundle(Server* s, const Cmd& c) {
  Query& q = *s->queries[c.q];
  const kpa_row_layout& L = q.layout;
  // windows touched, from the producer's event-time bounds
  const u64 lo_t = c.ts_base + c.ts_lo, hi_t = c.ts_base + c.ts_hi;
  u64 w_lo = lo_t >= q.origin ? (lo_t - q.origin) / q.win_len : 0;
  const u64 w_hi = hi_t >= q.origin ? (hi_t - q.origin) / q.win_len : 0;
  u32 si = 0;
  Bundle* b = nullptr;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    if (hi_t < q.origin || w_hi < q.next_close) {  // every row is late
      s->n_late += c.n;
      return true;
    }
    w_lo = std::max(w_lo, q.next_close);
    const u64 kbytes = rnd(c.n * 8) * 2;                                  // sorted keys | values
    const u64 rbytes = s->cfg.rows_in_host ? 0 : rnd(c.n * L.row_bytes);  // rows on the device
    // impact tag: High when the bundle feeds one of its query's two next
    // windows to close, Low when it feeds a later one
    const bool want_host = place_on_host(s, w_lo < q.next_close + 2);
    const bool never = (rbytes && !s->pool.fits_ever(rbytes, false)) ||
                       (!s->pool.fits_ever(kbytes + rbytes, false) &&
                        !(s->hmem && s->hpool.fits_ever(kbytes, false)));
    if (never) {
      fail_locked(s, KPA_EBUDGET, "a bundle can never fit the server's pools");
      return false;
    }
    bool waited = false;
    while (true) {
      if (s->stop) return false;
      // a free slot
      si = (u32)s->slots.size();
      for (u32 i = 0; i < s->slots.size(); ++i) {
        Slot& sl = s->slots[i];
        if (!sl.used || hipEventQuery(sl.last) == hipSuccess) {
          si = i;
          break;
        }
      }
      const bool rec_ok = !s->free_records.empty();
      void *mem = nullptr, *rmem = nullptr;
      bool on_host = false;
      if (si < s->slots.size() && rec_ok) {
        if (rbytes) rmem = s->pool.try_alloc(rbytes, false);
        if (!rbytes || rmem) {
          if (!want_host) mem = s->pool.try_alloc(kbytes, false);
          if (!mem && s->hmem) {  // placed on the host, or spilled from a full device pool
            mem = s->hpool.try_alloc(kbytes, false);
            on_host = mem != nullptr;
          }
          if (!mem && rmem) {
            s->pool.release(rmem, rbytes);
            rmem = nullptr;
          }
        }
      }
      if (mem) {
        s->stalled = false;
        b = new Bundle;
        b->q = c.q;
        b->side = c.side;
        b->n = c.n;
        b->w_lo = w_lo;
        b->n_win = (u32)(w_hi - w_lo + 1);
        b->block = mem;
        b->bytes = kbytes;
        b->on_host = on_host;
        b->rblock = rmem;
        b->rbytes = rbytes;
        b->keys = static_cast<u64*>(mem);
        b->vals = reinterpret_cast<u64*>(static_cast<char*>(mem) + rnd(c.n * 8));
        if (rmem) b->rows = static_cast<unsigned char*>(rmem);
        if (on_host) {
          s->n_host++;
          s->host_moved += 16 * c.n;  // the sorted KPA goes out over the host link
        }
        const u32 rec = s->free_records.back();
        s->free_records.pop_back();
        b->h_off = s->h_records + (u64)rec * RECORD_WORDS;
        b->done = take_event(s);
        b->refs = (int)b->n_win;
        s->live_bundles.insert(b);
        for (u64 w = w_lo; w <= w_hi; ++w) q.by_win[c.side][w].push_back(b);
        s->slots[si].used = true;
        s->n_bundles++;
        s->n_rows += c.n;
        s->rows_moved += c.n * L.row_bytes;  // the rows come in over the host link
        break;
      }
      if (!waited) {
        s->n_waits++;
        waited = true;
      }
      // back-pressure: wait for a close to free memory, or for a slot
      early_watermarks(s, c.q, w_lo);
      // stalled: memory or records are short and no close is queued or
      // running; only a close frees them, so only a watermark that the
      // producer has not sent yet can end the wait
      const bool stalled = si < s->slots.size() && s->closes_in == s->closes_done;
      if (stalled != s->stalled) {
        s->stalled = stalled;
        s->cv_space.notify_all();  // a blocked submit and drain look again
        s->cv_done.notify_all();
      }
      s->cv_space.wait_for(lk, std::chrono::microseconds(200));
    }
  }
  if (!b->done) {
    fail(s, KPA_EHIP, "event creation failed");
    return false;
  }
  Slot& sl = s->slots[si];
  unsigned char* dev_rows = b->rows ? b->rows : sl.staging;
  kpa_status rc = kpa_ingest_bundle(c.rows, c.n, &L, c.ts_base, dev_rows, sl.st);
  if (rc == KPA_OK)
    rc = kpa_partition_windows(dev_rows, c.n, &L, q.win_len, q.origin + w_lo * q.win_len, b->n_win,
                               0, sl.pkeys, sl.prids, sl.pvals, sl.win_off, sl.oob, sl.part_ws,
                               sl.part_ws_bytes, sl.st);
  // a KPA placed on the host is sorted into the slot's scratch and copied out
  u64* okeys = b->on_host ? sl.okeys : b->keys;
  u64* ovals = b->on_host ? sl.ovals : b->vals;
  if (rc == KPA_OK)
    rc = kpa_sort_segmented(sl.pkeys, sl.prids, okeys, sl.srids, sl.win_off, b->n_win, c.n,
                            KPA_SORT_RADIX, nullptr, nullptr, sl.sort_ws, sl.sort_ws_bytes, sl.st);
  if (rc == KPA_OK) {
    hipLaunchKernelGGL(k_gather_vals, dim3((u32)std::min<u64>(ceil_div(c.n, BLOCK), 2048)),
                       dim3(BLOCK), 0, sl.st, sl.srids, sl.pvals, sl.win_off + b->n_win, ovals);
    if (hipGetLastError() != hipSuccess) rc = KPA_EHIP;
  }
  if (rc == KPA_OK && b->on_host &&
      (hipMemcpyAsync(b->keys, okeys, c.n * 8, hipMemcpyDeviceToHost, sl.st) != hipSuccess ||
       hipMemcpyAsync(b->vals, ovals, c.n * 8, hipMemcpyDeviceToHost, sl.st) != hipSuccess))
    rc = KPA_EHIP;
  if (rc == KPA_OK &&
      (hipMemcpyAsync(b->h_off, sl.win_off, (b->n_win + 1) * sizeof(u64), hipMemcpyDeviceToHost,
                      sl.st) != hipSuccess ||
       hipMemcpyAsync(b->h_off + b->n_win + 1, sl.oob, sizeof(u64), hipMemcpyDeviceToHost,
                      sl.st) != hipSuccess ||
       hipEventRecord(b->done, sl.st) != hipSuccess || hipEventRecord(sl.last, sl.st) != hipSuccess))
    rc = KPA_EHIP;
  if (rc != KPA_OK) {
    fail(s, rc, "bundle launch failed");
    return false;
  }
  return true;
}

void run_watermark(Server* s, const Cmd& c) {
  std::lock_guard<std::mutex> lk(s->mu);
  close_windows(s, c);
}

// Applies a watermark: queues the close of every window that ends at or
// before it.  Caller holds the lock.
void close_windows(Server* s, const Cmd& c) {
  Query& q = *s->queries[c.q];
  if (q.have_wm && c.t <= q.wm) return;
  q.wm = c.t;
  q.have_wm = true;
  // windows [origin + w*W, origin + (w+1)*W) with end <= t close; only
  // windows that received rows produce a result
  if (c.t < q.origin) return;
  const u64 closable = (c.t - q.origin) / q.win_len;  // windows w < closable
  if (closable <= q.next_close) return;
  std::vector<u64> ws;
  for (int sd = 0; sd < q.sides; ++sd)
    for (auto it = q.by_win[sd].lower_bound(q.next_close);
         it != q.by_win[sd].end() && it->first < closable; ++it)
      ws.push_back(it->first);
  std::sort(ws.begin(), ws.end());
  ws.erase(std::unique(ws.begin(), ws.end()), ws.end());
  for (u64 w : ws) {
    CloseJob j;
    j.q = c.q;
    j.w = w;
    j.t_ingest = c.at;
    for (int sd = 0; sd < q.sides; ++sd) {
      auto it = q.by_win[sd].find(w);
      if (it != q.by_win[sd].end()) {
        j.runs[sd] = std::move(it->second);
        q.by_win[sd].erase(it);
      }
    }
    s->closes.push_back(std::move(j));
    s->closes_in++;
  }
  q.next_close = closable;
  s->cv_close.notify_all();
}

void dispatcher_main(Server* s) {
  if (hipSetDevice(s->device) != hipSuccess) {
    fail(s, KPA_EHIP, "hipSetDevice in dispatcher");
    return;
  }
  while (true) {
    Cmd c;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_cmd.wait(lk, [&] { return s->stop || !s->cmds.empty(); });
      if (s->stop) return;
      c = s->cmds.front();
      s->cmds.pop_front();
      s->cv_space.notify_all();  // a place in the pending queue
    }
    bool ok = true;
    if (c.kind == Cmd::BUNDLE)
      ok = run_bundle(s, c);
    else
      run_watermark(s, c);
    std::lock_guard<std::mutex> lk(s->mu);
    s->cmds_done++;
    s->cv_done.notify_all();
    if (!ok) return;
  }
}

// -------------------------------------------------------------- closer --

// Device memory of one close.  Only closes release pool memory (the bundles
// of a closed window, and a close's own buffers when it ends), so a close that
// finds too little free memory cannot wait for more: it reports the shortage
// and the server stops with KPA_EBUDGET.  The short waits cover the
// dispatcher, which may hold rows memory for a moment while it backs out of
// an admission.
struct CloseBufs {
  std::vector<std::pair<void*, u64>> held;
  Server* s;
  bool short_mem = false;  // the close needs more device memory than is free
  u64 asked = 0;           // bytes of the request that failed, and the close's total so far
  u64 total = 0;
  hipStream_t st;
  CloseBufs(Server* sv, hipStream_t stream) : s(sv), st(stream) {}
  void* take(u64 bytes) {
    std::unique_lock<std::mutex> lk(s->mu);
    for (int tries = 0; tries < 50; ++tries) {
      if (s->stop) return nullptr;
      void* p = s->pool.try_alloc(bytes, true);
      if (p) {
        held.emplace_back(p, bytes);
        total += bytes;
        s->close_bytes += bytes;
        return p;
      }
      s->cv_space.wait_for(lk, std::chrono::microseconds(200));
    }
    short_mem = true;
    asked = bytes;
    return nullptr;
  }
  ~CloseBufs() {
    // a close that fails part way may still have kernels in flight on them
    if (!held.empty()) (void)hipStreamSynchronize(st);
    std::lock_guard<std::mutex> lk(s->mu);
    for (auto& h : held) s->pool.release(h.first, h.second);
    s->close_bytes -= total;
    s->cv_space.notify_all();
  }
};

// Concatenates the window's runs of one side (keys, and their values) and
// merges them into one sorted KPA whose rids index the concatenated values.
// Returns the entry count, or -1 on failure.
long long merge_side(Server* s, CloseBufs& cb, const CloseJob& j, int side, u64** out_k,
                     u32** out_r, u64** out_v, hipStream_t st, u32* runs, u32* runs_host) {
  std::vector<u64> off{0};
  std::vector<std::pair<const Bundle*, std::pair<u64, u64>>> parts;
  u64 from_host = 0;
  for (const Bundle* b : j.runs[side]) {
    if (hipEventSynchronize(b->done) != hipSuccess) return -1;
    const u64 k = j.w - b->w_lo;
    const u64 a = b->h_off[k], e = b->h_off[k + 1];
    if (e > a) {
      parts.push_back({b, {a, e - a}});
      off.push_back(off.back() + (e - a));
      ++*runs;
      if (b->on_host) {
        ++*runs_host;
        from_host += 16 * (e - a);
      }
    }
  }
  if (from_host) {  // the host-pool runs come back over the host link
    std::lock_guard<std::mutex> lk(s->mu);
    s->host_moved += from_host;
  }
  const u64 n = off.back();
  *out_k = nullptr;
  *out_r = nullptr;
  *out_v = nullptr;
  if (n == 0) return 0;
  u64* ck = static_cast<u64*>(cb.take(n * 8));
  u32* cr = static_cast<u32*>(cb.take(n * 4));
  u64* cv = static_cast<u64*>(cb.take(n * 8));
  u64* mk = static_cast<u64*>(cb.take(n * 8));
  u32* mr = static_cast<u32*>(cb.take(n * 4));
  size_t wsb = 0;
  if (!ck || !cr || !cv || !mk || !mr || kpa_merge_runs_workspace_size(n, &wsb) != KPA_OK)
    return -1;
  void* ws = cb.take(wsb);
  if (!ws) return -1;
  for (size_t i = 0; i < parts.size(); ++i) {
    const Bundle* b = parts[i].first;
    const u64 a = parts[i].second.first, len = parts[i].second.second;
    const hipMemcpyKind kind = b->on_host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    if (hipMemcpyAsync(ck + off[i], b->keys + a, len * 8, kind, st) != hipSuccess ||
        hipMemcpyAsync(cv + off[i], b->vals + a, len * 8, kind, st) != hipSuccess)
      return -1;
  }
  hipLaunchKernelGGL(k_iota, dim3((u32)std::min<u64>(ceil_div(n, BLOCK), 4096)), dim3(BLOCK), 0,
                     st, cr, n);
  if (hipGetLastError() != hipSuccess) return -1;
  if (kpa_merge_runs(ck, cr, off.data(), (u32)parts.size(), mk, mr, ws, wsb, st) != KPA_OK)
    return -1;
  *out_k = mk;
  *out_r = mr;
  *out_v = cv;
  return (long long)n;
}

bool do_close(Server* s, const CloseJob& j, kpa_window_result* res, std::string* budget) {
  Query& q = *s->queries[j.q];
  hipStream_t st = s->close_st;
  CloseBufs cb(s, st);
  struct BudgetFlag {
    CloseBufs& cb;
    Server* s;
    const CloseJob& j;
    std::string* out;
    ~BudgetFlag() {
      if (!cb.short_mem) return;
      char msg[320];
      std::lock_guard<std::mutex> lk(s->mu);
      std::snprintf(msg, sizeof(msg),
                    "closing window %llu of query %u needs more device memory than is free "
                    "(%llu bytes held by the close, %llu more asked, %llu of %llu pool bytes in "
                    "use by open windows and the close)",
                    (unsigned long long)j.w, j.q, (unsigned long long)cb.total,
                    (unsigned long long)cb.asked, (unsigned long long)s->pool.used(),
                    (unsigned long long)s->pool.size());
      *out = msg;
    }
  } flag{cb, s, j, budget};
  std::memset(res, 0, sizeof(*res));
  res->query = j.q;
  res->kind = q.kind;
  res->window = j.w;
  u64* mk[2] = {nullptr, nullptr};
  u32* mr[2] = {nullptr, nullptr};
  u64* mv[2] = {nullptr, nullptr};
  long long n[2] = {0, 0};
  for (int sd = 0; sd < q.sides; ++sd) {
    n[sd] = merge_side(s, cb, j, sd, &mk[sd], &mr[sd], &mv[sd], st, &res->runs, &res->runs_host);
    if (n[sd] < 0) return false;
    res->rows[sd] = (u64)n[sd];
  }
  // per-key columns to hand to the caller (keep_groups): device arrays of
  // N entries each, the first G of them valid
  u64* cols[4] = {nullptr, nullptr, nullptr, nullptr};
  int ncols = 0;
  // small device results: [0..1] segment offsets side 0, [2..3] side 1,
  // [4] digest, [5] total, [6] groups / pairs, [7] sumprod, [8..9] scratch
  u64* small = static_cast<u64*>(cb.take(16 * sizeof(u64)));
  if (!small) return false;
  if (launch_fill_u64(small, 16, 0, st) != KPA_OK) return false;
  hipLaunchKernelGGL(k_set2, dim3(1), dim3(1), 0, st, small, (u64)0, (u64)n[0]);
  hipLaunchKernelGGL(k_set2, dim3(1), dim3(1), 0, st, small + 2, (u64)0, (u64)n[1]);
  if (hipGetLastError() != hipSuccess) return false;
  const kpa_row_layout V{8, 0, 0, 8, 0, 8};  // concatenated values read as 8-byte rows
  u64 host[8 + 2 * 10];
  std::memset(host, 0, sizeof(host));
  u32 n_top = 0;
  if (q.kind == KPA_Q_SUM && n[0] > 0) {
    const u64 N = (u64)n[0];
    u64* g = static_cast<u64*>(cb.take(4 * N * 8));
    size_t rwb = 0, twb = 0;
    if (!g || kpa_reduce_by_key_workspace_size(N, 1, &rwb) != KPA_OK ||
        kpa_topk_by_sum_workspace_size(N, 1, &twb) != KPA_OK)
      return false;
    void* rws = cb.take(rwb);
    void* tws = cb.take(twb);
    u64* top = static_cast<u64*>(cb.take(24 * 8));
    if (!rws || !tws || !top) return false;
    u64 *gk = g, *gc = g + N, *gs = g + 2 * N, *gm = g + 3 * N;
    if (kpa_reduce_by_key(mk[0], mr[0], small, 1, N, mv[0], &V, gk, gc, gs, gm, nullptr,
                          small + 8, rws, rwb, st) != KPA_OK ||
        kpa_topk_by_sum(gk, gs, small + 8, 1, N, 10, top, top + 10,
                        reinterpret_cast<u32*>(top + 20), tws, twb, st) != KPA_OK)
      return false;
    cols[0] = gk, cols[1] = gc, cols[2] = gs, cols[3] = gm;
    ncols = 4;
    hipLaunchKernelGGL(k_digest, dim3(256), dim3(BLOCK), 0, st, gk, gc, gs, gm, small + 9,
                       small + 4);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(host + 8, top, 20 * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(&n_top, top + 20, 4, hipMemcpyDeviceToHost, st) != hipSuccess)
      return false;
  } else if (q.kind == KPA_Q_MEDIAN && n[0] > 0) {
    const u64 N = (u64)n[0];
    u64* g = static_cast<u64*>(cb.take(2 * N * 8));
    size_t mwb = 0;
    if (!g || kpa_median_by_key_workspace_size(N, 1, &mwb) != KPA_OK) return false;
    void* mws = cb.take(mwb);
    if (!mws) return false;
    if (kpa_median_by_key(mk[0], mr[0], small, 1, N, mv[0], &V, g, g + N, small + 8, nullptr,
                          nullptr, mws, mwb, st) != KPA_OK)
      return false;
    cols[0] = g, cols[1] = g + N;
    ncols = 2;
    hipLaunchKernelGGL(k_digest, dim3(256), dim3(BLOCK), 0, st, g, g + N, nullptr, nullptr,
                       small + 9, small + 4);
    if (hipGetLastError() != hipSuccess) return false;
  } else if (q.kind == KPA_Q_JOIN && n[0] > 0 && n[1] > 0) {
    size_t jwb = 0;
    if (kpa_join_workspace_size((u64)n[0], (u64)n[1], 1, &jwb) != KPA_OK) return false;
    void* jws = cb.take(jwb);
    if (!jws) return false;
    if (kpa_join(mk[0], mr[0], small, (u64)n[0], mk[1], mr[1], small + 2, (u64)n[1], 1,
                 mv[0], mv[1], &V, small + 6, small + 7, nullptr, 0, nullptr,
                 jws, jwb, st) != KPA_OK)
      return false;
  }
  if (hipMemcpyAsync(host, small + 4, 4 * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(host + 4, small + 8, 2 * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return false;
  // host: [0] digest, [1] total, [2] pairs, [3] sumprod, [4] gseg_off[0], [5] groups
  if (q.kind == KPA_Q_JOIN) {
    res->groups = host[2];
    res->total = host[3];
  } else {
    res->groups = host[5];
    res->total = q.kind == KPA_Q_SUM ? host[1] : 0;
    res->digest = host[0];
  }
  if (q.kind == KPA_Q_SUM) {
    res->n_top = std::min<u32>(n_top, 10);
    for (u32 i = 0; i < res->n_top; ++i) {
      res->top_key[i] = host[8 + i];
      res->top_sum[i] = host[18 + i];
    }
  }
  if (s->cfg.keep_groups && ncols && res->groups) {
    const u64 G = res->groups;
    uint64_t* h = new (std::nothrow) uint64_t[G * ncols];
    if (!h) return false;
    for (int c = 0; c < ncols; ++c)
      if (hipMemcpyAsync(h + c * G, cols[c], G * 8, hipMemcpyDeviceToHost, st) != hipSuccess) {
        delete[] h;
        return false;
      }
    if (hipStreamSynchronize(st) != hipSuccess) {
      delete[] h;
      return false;
    }
    res->groups_data = h;
    res->groups_words = G * ncols;
    std::lock_guard<std::mutex> lk(s->mu);
    s->groups_out.insert(h);
  }
  return true;
}

void closer_main(Server* s) {
  if (hipSetDevice(s->device) != hipSuccess) {
    fail(s, KPA_EHIP, "hipSetDevice in closer");
    return;
  }
  while (true) {
    CloseJob j;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_close.wait(lk, [&] { return s->stop || !s->closes.empty(); });
      if (s->stop) return;
      j = std::move(s->closes.front());
      s->closes.pop_front();
    }
    kpa_window_result r;
    std::string budget;
    if (!do_close(s, j, &r, &budget)) {
      if (!budget.empty())
        fail(s, KPA_EBUDGET, budget.c_str());
      else
        fail(s, KPA_EHIP, "window close failed");
      return;
    }
    const auto now = Clock::now();
    r.latency_ms = std::chrono::duration<double, std::milli>(now - j.t_ingest).count();
    std::lock_guard<std::mutex> lk(s->mu);
    for (int sd = 0; sd < 2; ++sd)
      for (Bundle* b : j.runs[sd])
        if (--b->refs == 0) {
          s->n_late += b->h_off[b->n_win + 1];  // rows outside the bundle's open windows
          release_bundle(s, b);
        }
    s->results.push_back(r);
    s->lat_ms.push_back(r.latency_ms);
    s->t_last = now;
    s->closes_done++;
    s->cv_space.notify_all();
    s->cv_done.notify_all();
  }
}

// Every monitor_ms: device-pool use, host-link traffic of the interval and
// the current output delay; the knob moves (balanced placement) and the
// sample is kept for kpa_server_trace.
constexpr size_t TRACE_CAP = 65536;

void monitor_main(Server* s) {
  u64 last_moved = 0;
  double bw = 0.0;  // host-link use, smoothed over about 100 ms
  Clock::time_point last = Clock::now();
  std::unique_lock<std::mutex> lk(s->mu);
  while (!s->stop) {
    s->cv_done.wait_for(lk, std::chrono::milliseconds(s->cfg.monitor_ms));
    if (s->stop) return;
    const Clock::time_point now = Clock::now();
    const double dt = std::chrono::duration<double>(now - last).count();
    if (dt <= 0) continue;
    // capacity: the pool outside the close reserve, against what bundles
    // hold (close scratch is urgent work from the reserve)
    const double cap = (double)(s->pool.size() - s->pool.size() / 100 * s->cfg.reserve_pct);
    const u64 held = s->pool.used() - std::min(s->pool.used(), s->close_bytes);
    const double hbm = cap > 0 ? std::min(1.0, (double)held / cap) : 1.0;
    // link: rows in at ingest plus host-pool KPAs out and back
    const u64 moved_now = s->host_moved + s->rows_moved;
    const u64 moved = moved_now - last_moved;
    const double inst =
        s->host_bw > 0 ? std::min(1.0, (double)moved / (dt * s->host_bw * 1e9)) : 0.0;
    const double a = dt / (dt + 0.1);
    bw += a * (inst - bw);
    double delay = 0;
    const size_t nl = s->lat_ms.size();
    for (size_t i = nl > 16 ? nl - 16 : 0; i < nl; ++i) delay = std::max(delay, s->lat_ms[i]);
    if (s->cfg.placement == KPA_PLACE_BALANCED)
      (void)kpa_balance_knob_update(&s->k_low, &s->k_high, hbm, bw, delay,
                                    s->cfg.target_delay_ms);
    last = now;
    last_moved = moved_now;
    if (!s->started) continue;
    kpa_monitor_sample m;
    m.t_s = std::chrono::duration<double>(now - s->t_first).count();
    m.hbm_util = hbm;
    m.bw_util = bw;
    m.k_low = s->k_low;
    m.k_high = s->k_high;
    m.delay_ms = delay;
    m.hbm_bytes = s->pool.used();
    m.host_bytes = s->hmem ? s->hpool.used() : 0;
    m.waits = s->n_waits;
    m.bundles_host = s->n_host;
    if (s->trace.size() >= TRACE_CAP) s->trace.erase(s->trace.begin(), s->trace.begin() + TRACE_CAP / 2);
    s->trace.push_back(m);
  }
}

kpa_status check_server_config(const kpa_server_config* c) {
  KPA_REQUIRE(c != nullptr, KPA_EINVAL, "config is null");
  KPA_REQUIRE(c->slots >= 1 && c->slots <= 64, KPA_EINVAL, "slots must be in [1, 64]");
  KPA_REQUIRE(c->max_bundle_rows >= 1 && c->max_bundle_rows < (1ull << 30), KPA_EINVAL,
              "max_bundle_rows must be in [1, 2^30)");
  KPA_REQUIRE(c->max_row_bytes >= 8 && c->max_row_bytes <= 256 && c->max_row_bytes % 8 == 0,
              KPA_EINVAL, "max_row_bytes must be a multiple of 8 in [8, 256]");
  KPA_REQUIRE(c->max_pending >= 1, KPA_EINVAL, "max_pending must be >= 1");
  KPA_REQUIRE(c->reserve_pct <= 90, KPA_EINVAL, "reserve_pct must be at most 90");
  KPA_REQUIRE(c->max_live_bundles >= 1, KPA_EINVAL, "max_live_bundles must be >= 1");
  KPA_REQUIRE(c->placement <= KPA_PLACE_HOST, KPA_EINVAL, "bad placement");
  KPA_REQUIRE(c->placement == KPA_PLACE_DEVICE || c->host_pool_bytes > 0, KPA_EINVAL,
              "host placement needs a host pool (host_pool_bytes > 0)");
  KPA_REQUIRE(c->monitor_ms >= 1 && c->monitor_ms <= 60000, KPA_EINVAL,
              "monitor_ms must be in [1, 60000]");
  KPA_REQUIRE(c->target_delay_ms > 0 && c->host_bw_gbs >= 0, KPA_EINVAL,
              "target_delay_ms must be positive and host_bw_gbs not negative");
  return KPA_OK;
}

void teardown(Server* s) {
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_cmd.notify_all();
    s->cv_space.notify_all();
    s->cv_close.notify_all();
    s->cv_done.notify_all();
  }
  if (s->dispatcher.joinable()) s->dispatcher.join();
  if (s->closer.joinable()) s->closer.join();
  if (s->monitor.joinable()) s->monitor.join();
  for (const uint64_t* g : s->groups_out) delete[] g;
  s->groups_out.clear();
  (void)hipSetDevice(s->device);
  for (auto& sl : s->slots) {
    if (sl.st) (void)hipStreamSynchronize(sl.st);
  }
  if (s->close_st) (void)hipStreamSynchronize(s->close_st);
  for (Bundle* b : s->live_bundles) {
    if (b->done) s->event_pool.push_back(b->done);
    delete b;
  }
  s->live_bundles.clear();
  for (auto& sl : s->slots) {
    if (sl.last) (void)hipEventDestroy(sl.last);
    if (sl.st) (void)hipStreamDestroy(sl.st);
  }
  for (hipEvent_t e : s->event_pool) (void)hipEventDestroy(e);
  if (s->close_st) (void)hipStreamDestroy(s->close_st);
  if (s->h_records) (void)hipHostFree(s->h_records);
  if (s->hmem) (void)hipHostFree(s->hmem);
  if (s->mem) (void)hipFree(s->mem);
}

}  // namespace
}  // namespace kpa

using namespace kpa;

extern "C" {

kpa_status kpa_ingest_bundle(const void* host_rows, uint64_t n, const kpa_row_layout* layout,
                             uint64_t ts_add, void* dev_rows, hipStream_t stream) {
  clear_error();
  KPA_CHECK(check_layout(layout, false, ts_add != 0));
  if (n == 0) return KPA_OK;
  KPA_REQUIRE(host_rows && dev_rows, KPA_EINVAL, "null pointer");
  KPA_REQUIRE(aligned(dev_rows, 16), KPA_EINVAL, "misaligned device rows");
  KPA_HIP(hipMemcpyAsync(dev_rows, host_rows, n * layout->row_bytes, hipMemcpyHostToDevice,
                         stream));
  if (ts_add)
    KPA_LAUNCH("ingest_rebase", k_add_ts, dim3((u32)std::min<u64>(ceil_div(n, BLOCK), 4096)),
               dim3(BLOCK), 0, stream, static_cast<unsigned char*>(dev_rows), n,
               layout->row_bytes, layout->ts_off, layout->ts_w, ts_add);
  return KPA_OK;
}

kpa_status kpa_server_config_default(kpa_server_config* cfg) {
  clear_error();
  KPA_REQUIRE(cfg != nullptr, KPA_EINVAL, "config is null");
  cfg->budget_bytes = 64ull << 30;
  cfg->slots = 8;
  cfg->rows_in_host = 0;
  cfg->max_bundle_rows = 1u << 20;
  cfg->max_row_bytes = 32;
  cfg->max_pending = 256;
  cfg->reserve_pct = 25;
  cfg->max_live_bundles = 1u << 16;
  cfg->host_pool_bytes = 0;
  cfg->placement = KPA_PLACE_DEVICE;
  cfg->monitor_ms = 10;
  cfg->target_delay_ms = 1000.0;
  cfg->host_bw_gbs = 0.0;
  cfg->keep_groups = 0;
  cfg->seed = 1;
  return KPA_OK;
}

kpa_status kpa_balance_knob_update(double* k_low, double* k_high, double hbm_util,
                                   double bw_util, double delay_ms, double target_ms) {
  clear_error();
  KPA_REQUIRE(k_low && k_high, KPA_EINVAL, "null knob");
  constexpr double DELTA = 0.05, SLACK = 0.1, HEADROOM = 0.9;
  double d = 0;
  if (hbm_util > bw_util + SLACK) d = -DELTA;       // capacity is short: toward the host
  else if (bw_util > hbm_util + SLACK) d = DELTA;   // the host link is short: toward HBM
  if (d == 0) return KPA_OK;
  const bool low_at_end = d < 0 ? *k_low <= 0.0 : *k_low >= 1.0;
  if (!low_at_end) {
    *k_low = std::min(1.0, std::max(0.0, *k_low + d));
  } else if (delay_ms <= HEADROOM * target_ms) {
    *k_high = std::min(1.0, std::max(0.0, *k_high + d));
  }
  return KPA_OK;
}

kpa_status kpa_server_create(const kpa_server_config* cfg, kpa_server* out) {
  clear_error();
  KPA_REQUIRE(out != nullptr, KPA_EINVAL, "out is null");
  *out = nullptr;
  KPA_CHECK(check_server_config(cfg));
  // per-slot scratch, sized for the largest bundle
  const u64 mb = cfg->max_bundle_rows;
  size_t part_ws = 0, sort_ws = 0;
  KPA_CHECK(kpa_partition_windows_workspace_size(mb, MAX_BUNDLE_WINDOWS, &part_ws));
  KPA_CHECK(kpa_sort_workspace_size(mb, MAX_BUNDLE_WINDOWS, KPA_SORT_RADIX, &sort_ws));
  const bool host_tier = cfg->host_pool_bytes > 0;
  const u64 slot_bytes = rnd(mb * 8) + rnd(mb * 4) + rnd(mb * 8) + rnd(mb * 4) +
                         rnd((MAX_BUNDLE_WINDOWS + 2) * 8) +
                         rnd(part_ws) + rnd(sort_ws) +
                         (cfg->rows_in_host ? rnd(mb * cfg->max_row_bytes) : 0) +
                         (host_tier ? 2 * rnd(mb * 8) : 0);
  const u64 fixed = slot_bytes * cfg->slots;
  KPA_REQUIRE(cfg->budget_bytes > fixed + (64ull << 20), KPA_EBUDGET,
              "budget of %llu bytes does not cover the slots' scratch (%llu bytes)",
              (unsigned long long)cfg->budget_bytes, (unsigned long long)fixed);
  {
    // the largest bundle must be admissible: its rows (when kept on the
    // device) and its KPA in the device pool, or the KPA in the host pool
    const u64 pool_bytes = cfg->budget_bytes - fixed;
    const u64 normal = pool_bytes - pool_bytes / 100 * cfg->reserve_pct;
    const u64 rbytes = cfg->rows_in_host ? 0 : rnd(mb * cfg->max_row_bytes);
    const u64 kbytes = 2 * rnd(mb * 8);
    const bool fits = rbytes + kbytes <= normal ||
                      (host_tier && rbytes <= normal && kbytes <= cfg->host_pool_bytes);
    KPA_REQUIRE(fits, KPA_EBUDGET,
                "a bundle of %llu rows needs %llu bytes of pool memory; the budget leaves %llu "
                "(the rest is scratch and the close reserve)",
                (unsigned long long)mb, (unsigned long long)(rbytes + kbytes),
                (unsigned long long)normal);
  }
  std::unique_ptr<Server> s(new (std::nothrow) Server);
  KPA_REQUIRE(s != nullptr, KPA_EINVAL, "out of host memory");
  s->cfg = *cfg;
  KPA_HIP(hipGetDevice(&s->device));
  hipError_t e = hipMalloc(&s->mem, cfg->budget_bytes);
  if (e != hipSuccess) {
    s->mem = nullptr;
    KPA_REQUIRE(false, KPA_EBUDGET, "cannot allocate the %llu-byte budget: %s",
                (unsigned long long)cfg->budget_bytes, hipGetErrorString(e));
  }
  // slot scratch at the start, the rest is the pool
  char* p = s->mem;
  s->slots.resize(cfg->slots);
  for (auto& sl : s->slots) {
    sl.pkeys = reinterpret_cast<u64*>(p);
    p += rnd(mb * 8);
    sl.prids = reinterpret_cast<u32*>(p);
    p += rnd(mb * 4);
    sl.pvals = reinterpret_cast<u64*>(p);
    p += rnd(mb * 8);
    sl.srids = reinterpret_cast<u32*>(p);
    p += rnd(mb * 4);
    sl.win_off = reinterpret_cast<u64*>(p);
    sl.oob = sl.win_off + MAX_BUNDLE_WINDOWS + 1;
    p += rnd((MAX_BUNDLE_WINDOWS + 2) * 8);
    sl.part_ws = p;
    sl.part_ws_bytes = part_ws;
    p += rnd(part_ws);
    sl.sort_ws = p;
    sl.sort_ws_bytes = sort_ws;
    p += rnd(sort_ws);
    if (cfg->rows_in_host) {
      sl.staging = reinterpret_cast<unsigned char*>(p);
      p += rnd(mb * cfg->max_row_bytes);
    }
    if (host_tier) {
      sl.okeys = reinterpret_cast<u64*>(p);
      p += rnd(mb * 8);
      sl.ovals = reinterpret_cast<u64*>(p);
      p += rnd(mb * 8);
    }
  }
  const u64 pool_bytes = cfg->budget_bytes - (u64)(p - s->mem);
  s->pool.init(p, pool_bytes, pool_bytes / 100 * cfg->reserve_pct);
  struct Guard {
    Server* s;
    bool armed = true;
    ~Guard() {
      if (armed) teardown(s);
    }
  } guard{s.get()};
  for (auto& sl : s->slots) {
    KPA_HIP(hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking));
    KPA_HIP(hipEventCreateWithFlags(&sl.last, hipEventDisableTiming));
  }
  KPA_HIP(hipStreamCreateWithFlags(&s->close_st, hipStreamNonBlocking));
  KPA_HIP(hipHostMalloc(reinterpret_cast<void**>(&s->h_records),
                        (u64)cfg->max_live_bundles * RECORD_WORDS * sizeof(u64),
                        hipHostMallocDefault));
  s->free_records.reserve(cfg->max_live_bundles);
  for (u32 i = cfg->max_live_bundles; i > 0; --i) s->free_records.push_back(i - 1);
  s->rng = 0x5851F42D4C957F2Dull ^ ((u64)cfg->seed << 17);
  if (host_tier) {
    const hipError_t he = hipHostMalloc(reinterpret_cast<void**>(&s->hmem), cfg->host_pool_bytes,
                                        hipHostMallocDefault);
    if (he != hipSuccess) {
      s->hmem = nullptr;
      KPA_REQUIRE(false, KPA_EBUDGET, "cannot allocate the %llu-byte host pool: %s",
                  (unsigned long long)cfg->host_pool_bytes, hipGetErrorString(he));
    }
    s->hpool.init(s->hmem, cfg->host_pool_bytes, 0);
    s->host_bw = cfg->host_bw_gbs;
    if (s->host_bw <= 0) {
      // what a pinned host-to-device copy moves per second on this machine
      const u64 probe = std::min<u64>(cfg->host_pool_bytes, 64ull << 20) / ALIGN * ALIGN;
      hipEvent_t e0 = nullptr, e1 = nullptr;
      KPA_HIP(hipEventCreate(&e0));
      KPA_HIP(hipEventCreate(&e1));
      float ms = 0;
      hipError_t pe = hipMemcpyAsync(p, s->hmem, probe, hipMemcpyHostToDevice,
                                     s->close_st);
      if (pe == hipSuccess) pe = hipEventRecord(e0, s->close_st);
      if (pe == hipSuccess)
        pe = hipMemcpyAsync(p, s->hmem, probe, hipMemcpyHostToDevice,
                            s->close_st);
      if (pe == hipSuccess) pe = hipEventRecord(e1, s->close_st);
      if (pe == hipSuccess) pe = hipEventSynchronize(e1);
      if (pe == hipSuccess) pe = hipEventElapsedTime(&ms, e0, e1);
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      KPA_HIP(pe);
      s->host_bw = ms > 0 ? (double)probe / (ms * 1e-3) / 1e9 : 50.0;
    }
  }
  Server* raw = s.get();
  s->dispatcher = std::thread(dispatcher_main, raw);
  s->closer = std::thread(closer_main, raw);
  s->monitor = std::thread(monitor_main, raw);
  guard.armed = false;
  *out = s.release();
  return KPA_OK;
}

kpa_status kpa_server_add_query(kpa_server s, kpa_query_kind kind, const kpa_row_layout* layout,
                                uint64_t win_len, uint64_t win_origin, uint32_t* qid) {
  clear_error();
  KPA_REQUIRE(s != nullptr && qid != nullptr, KPA_EINVAL, "null argument");
  KPA_REQUIRE(kind == KPA_Q_SUM || kind == KPA_Q_MEDIAN || kind == KPA_Q_JOIN, KPA_EINVAL,
              "bad query kind");
  KPA_CHECK(check_layout(layout, true, true));
  KPA_REQUIRE(layout->row_bytes <= s->cfg.max_row_bytes, KPA_EINVAL,
              "row_bytes exceeds the server's max_row_bytes");
  KPA_REQUIRE(win_len >= 1, KPA_EINVAL, "win_len must be >= 1");
  std::unique_ptr<Query> q(new Query);
  q->kind = (u32)kind;
  q->layout = *layout;
  q->win_len = win_len;
  q->origin = win_origin;
  q->sides = kind == KPA_Q_JOIN ? 2 : 1;
  std::lock_guard<std::mutex> lk(s->mu);
  KPA_REQUIRE(s->failed == KPA_OK, s->failed, "server failed: %s", s->fail_msg.c_str());
  *qid = (u32)s->queries.size();
  s->queries.push_back(std::move(q));
  return KPA_OK;
}

kpa_status kpa_server_submit(kpa_server s, uint32_t qid, uint32_t side, const void* rows,
                             uint64_t n, uint64_t ts_base, uint64_t ts_lo, uint64_t ts_hi,
                             int32_t blocking) {
  clear_error();
  KPA_REQUIRE(s != nullptr, KPA_EINVAL, "server is null");
  if (n == 0) return KPA_OK;
  KPA_REQUIRE(rows != nullptr, KPA_EINVAL, "rows is null");
  KPA_REQUIRE(n <= s->cfg.max_bundle_rows, KPA_EINVAL, "bundle larger than max_bundle_rows");
  KPA_REQUIRE(ts_lo <= ts_hi, KPA_EINVAL, "ts_lo > ts_hi");
  std::unique_lock<std::mutex> lk(s->mu);
  KPA_REQUIRE(s->failed == KPA_OK, s->failed, "server failed: %s", s->fail_msg.c_str());
  KPA_REQUIRE(qid < s->queries.size(), KPA_EINVAL, "unknown query");
  const Query& q = *s->queries[qid];
  KPA_REQUIRE((int)side < q.sides, KPA_EINVAL, "bad side for this query");
  const u64 lo_t = ts_base + ts_lo, hi_t = ts_base + ts_hi;
  if (hi_t >= q.origin) {
    const u64 w_lo = lo_t >= q.origin ? (lo_t - q.origin) / q.win_len : 0;
    const u64 w_hi = (hi_t - q.origin) / q.win_len;
    KPA_REQUIRE(w_hi - w_lo < MAX_BUNDLE_WINDOWS, KPA_EINVAL,
                "a bundle may span at most %u windows", MAX_BUNDLE_WINDOWS);
  }
  while (s->cmds.size() >= s->cfg.max_pending) {
    if (!blocking) {
      KPA_REQUIRE(false, KPA_EBUDGET, "pending queue full (back-pressure)");
    }
    if (s->stalled) {
      // a watermark sent meanwhile from another thread is applied within
      // the dispatcher's next polls
      s->cv_space.wait_for(lk, std::chrono::milliseconds(5));
      KPA_REQUIRE(!s->stalled || s->cmds.size() < s->cfg.max_pending || s->failed != KPA_OK,
                  KPA_EBUDGET,
                  "pending queue full and the server stalled: the open windows hold all of the "
                  "pool memory or bundle records, so only a later watermark can free them");
    } else {
      s->cv_space.wait(lk);
    }
    KPA_REQUIRE(s->failed == KPA_OK, s->failed, "server failed: %s", s->fail_msg.c_str());
  }
  Cmd c;
  c.kind = Cmd::BUNDLE;
  c.q = qid;
  c.side = side;
  c.rows = rows;
  c.n = n;
  c.ts_base = ts_base;
  c.ts_lo = ts_lo;
  c.ts_hi = ts_hi;
  c.at = Clock::now();
  if (!s->started) {
    s->started = true;
    s->t_first = c.at;
  }
  s->cmds.push_back(c);
  s->cmds_in++;
  s->cv_cmd.notify_all();
  return KPA_OK;
}

kpa_status kpa_server_watermark(kpa_server s, uint32_t qid, uint64_t t) {
  clear_error();
  KPA_REQUIRE(s != nullptr, KPA_EINVAL, "server is null");
  std::lock_guard<std::mutex> lk(s->mu);
  KPA_REQUIRE(s->failed == KPA_OK, s->failed, "server failed: %s", s->fail_msg.c_str());
  KPA_REQUIRE(qid < s->queries.size(), KPA_EINVAL, "unknown query");
  Cmd c;
  c.kind = Cmd::WATERMARK;
  c.q = qid;
  c.t = t;
  c.at = Clock::now();
  s->cmds.push_back(c);  // watermarks are never refused
  s->cmds_in++;
  s->cv_cmd.notify_all();
  return KPA_OK;
}

kpa_status kpa_server_poll(kpa_server s, kpa_window_result* out, int32_t* got,
                           int32_t timeout_ms) {
  clear_error();
  KPA_REQUIRE(s != nullptr && out != nullptr && got != nullptr, KPA_EINVAL, "null argument");
  *got = 0;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->results.empty() && timeout_ms > 0)
    s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms),
                        [&] { return !s->results.empty() || s->failed != KPA_OK; });
  if (!s->results.empty()) {
    *out = s->results.front();
    s->results.pop_front();
    *got = 1;
    return KPA_OK;
  }
  KPA_REQUIRE(s->failed == KPA_OK, s->failed, "server failed: %s", s->fail_msg.c_str());
  return KPA_OK;
}

kpa_status kpa_server_drain(kpa_server s, int32_t timeout_ms) {
  clear_error();
  KPA_REQUIRE(s != nullptr, KPA_EINVAL, "server is null");
  std::unique_lock<std::mutex> lk(s->mu);
  auto done = [&] {
    return s->failed != KPA_OK ||
           (s->cmds_done == s->cmds_in && s->closes_done == s->closes_in);
  };
  auto idle = [&] { return done() || s->stalled; };
  const auto deadline = Clock::now() + std::chrono::milliseconds(std::max(timeout_ms, 0));
  while (true) {
    const bool ok = timeout_ms < 0 ? (s->cv_done.wait(lk, idle), true)
                                   : s->cv_done.wait_until(lk, deadline, idle);
    KPA_REQUIRE(s->failed == KPA_OK, s->failed, "server failed: %s", s->fail_msg.c_str());
    KPA_REQUIRE(ok, KPA_ETIMEOUT, "drain timed out (work still pending)");
    if (done()) return KPA_OK;
    // stalled: a watermark sent meanwhile from another thread is applied
    // within the dispatcher's next polls
    s->cv_done.wait_for(lk, std::chrono::milliseconds(5), [&] { return done() || !s->stalled; });
    KPA_REQUIRE(s->failed == KPA_OK, s->failed, "server failed: %s", s->fail_msg.c_str());
    KPA_REQUIRE(done() || !s->stalled, KPA_EBUDGET,
                "the server stalled: the open windows hold all of the pool memory or bundle "
                "records, and no queued watermark closes one of them");
  }
}

kpa_status kpa_server_stats(kpa_server s, kpa_server_statistics* out) {
  clear_error();
  KPA_REQUIRE(s != nullptr && out != nullptr, KPA_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(out, 0, sizeof(*out));
  out->bundles = s->n_bundles;
  out->rows = s->n_rows;
  out->late_rows = s->n_late;
  out->windows_closed = s->closes_done;
  out->backpressure_waits = s->n_waits;
  out->pool_peak_bytes = s->pool.peak();
  out->pool_bytes = s->pool.used();
  std::vector<double> l = s->lat_ms;
  if (!l.empty()) {
    std::sort(l.begin(), l.end());
    auto pct = [&](double p) {
      const size_t i = (size_t)std::min<double>((double)l.size() - 1, p * (double)(l.size() - 1) + 0.5);
      return l[i];
    };
    out->p50_ms = pct(0.50);
    out->p99_ms = pct(0.99);
    out->max_ms = l.back();
  }
  if (s->started) {
    const auto end = s->closes_done ? s->t_last : Clock::now();
    out->elapsed_s = std::chrono::duration<double>(end - s->t_first).count();
    if (out->elapsed_s > 0) out->mrec_per_s = (double)s->n_rows / out->elapsed_s / 1e6;
  }
  out->bundles_on_host = s->n_host;
  out->host_pool_bytes = s->hmem ? s->hpool.used() : 0;
  out->host_pool_peak_bytes = s->hmem ? s->hpool.peak() : 0;
  out->k_low = s->k_low;
  out->k_high = s->k_high;
  out->host_bw_gbs = s->host_bw;
  return KPA_OK;
}

kpa_status kpa_server_release_groups(kpa_server s, const uint64_t* groups_data) {
  clear_error();
  KPA_REQUIRE(s != nullptr, KPA_EINVAL, "server is null");
  if (!groups_data) return KPA_OK;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->groups_out.find(groups_data);
  KPA_REQUIRE(it != s->groups_out.end(), KPA_EINVAL, "not a result of this server");
  delete[] *it;
  s->groups_out.erase(it);
  return KPA_OK;
}

kpa_status kpa_server_trace(kpa_server s, kpa_monitor_sample* out, uint32_t cap, uint32_t* n) {
  clear_error();
  KPA_REQUIRE(s != nullptr && n != nullptr && (cap == 0 || out != nullptr), KPA_EINVAL,
              "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  const u32 m = (u32)std::min<size_t>(cap, s->trace.size());
  for (u32 i = 0; i < m; ++i) out[i] = s->trace[i];
  *n = m;
  return KPA_OK;
}

kpa_status kpa_server_destroy(kpa_server s) {
  clear_error();
  if (!s) return KPA_OK;
  teardown(s);
  delete s;
  return KPA_OK;
}

}  // extern "C"
