// Optional per-kernel timing with HIP events recorded around each launch on
// the launch's own stream.  Off by default; when off, the hooks cost one
// relaxed load.
#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "kpa_internal.hpp"

namespace kpa {

namespace {
struct Rec {
  const char* name;
  hipEvent_t a, b;
};
std::atomic<int> g_on{0};
std::mutex g_mu;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
std::map<std::string, std::pair<uint64_t, double>> g_sum;

hipEvent_t take_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

bool prof_enabled() { return g_on.load(std::memory_order_relaxed) != 0; }

int prof_begin(const char* name, hipStream_t st) {
  if (!g_on.load(std::memory_order_relaxed)) return -1;
  std::lock_guard<std::mutex> lk(g_mu);
  Rec r{name, take_event(), take_event()};
  if (!r.a || !r.b) return -1;
  if (hipEventRecord(r.a, st) != hipSuccess) return -1;
  g_recs.push_back(r);
  return (int)g_recs.size() - 1;
}

void prof_end(int slot, hipStream_t st) {
  if (slot < 0) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (slot < (int)g_recs.size()) (void)hipEventRecord(g_recs[slot].b, st);
}

}  // namespace kpa

using namespace kpa;

extern "C" {

kpa_status kpa_profile_enable(int32_t on) {
  clear_error();
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& r : g_recs) {
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
  g_sum.clear();
  g_on.store(on ? 1 : 0);
  return KPA_OK;
}

kpa_status kpa_profile_collect(void) {
  clear_error();
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& r : g_recs) {
    KPA_HIP(hipEventSynchronize(r.b));
    float ms = 0.f;
    KPA_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    auto& s = g_sum[r.name];
    s.first += 1;
    s.second += ms;
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
  return KPA_OK;
}

kpa_status kpa_profile_get(const char* name, uint64_t* launches, double* total_ms) {
  clear_error();
  KPA_REQUIRE(name && launches && total_ms, KPA_EINVAL, "null pointer");
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_sum.find(name);
  *launches = it == g_sum.end() ? 0 : it->second.first;
  *total_ms = it == g_sum.end() ? 0.0 : it->second.second;
  return KPA_OK;
}

kpa_status kpa_profile_names(char* buf, size_t len) {
  clear_error();
  KPA_REQUIRE(buf && len, KPA_EINVAL, "null buffer");
  std::lock_guard<std::mutex> lk(g_mu);
  std::string s;
  for (auto& kv : g_sum) {
    if (!s.empty()) s += ",";
    s += kv.first;
  }
  KPA_REQUIRE(s.size() < len, KPA_ECAPACITY, "buffer too small");
  std::memcpy(buf, s.c_str(), s.size() + 1);
  return KPA_OK;
}

}  // extern "C"
