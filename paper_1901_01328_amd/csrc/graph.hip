// Capture of a sequence of library calls into a HIP graph, replayed with one
// launch.  Every launch of the library sizes its grid from host-side
// capacities and reads actual sizes from device memory, and no call
// allocates, copies to the host or clears memory with a runtime memset, so a
// captured sequence stays valid for any input of the same capacities.
#include "kpa_internal.hpp"

struct kpa_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

using namespace kpa;

extern "C" {

kpa_status kpa_graph_begin(hipStream_t stream) {
  clear_error();
  KPA_REQUIRE(stream != nullptr, KPA_EINVAL, "the null stream cannot be captured");
  KPA_REQUIRE(!prof_enabled(), KPA_EINVAL, "disable per-kernel timing before capturing");
  KPA_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeRelaxed));
  return KPA_OK;
}

kpa_status kpa_graph_end(hipStream_t stream, kpa_graph* out) {
  clear_error();
  KPA_REQUIRE(stream != nullptr && out != nullptr, KPA_EINVAL, "null stream or output");
  *out = nullptr;
  hipGraph_t g = nullptr;
  KPA_HIP(hipStreamEndCapture(stream, &g));
  hipGraphExec_t e = nullptr;
  const hipError_t rc = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
  if (rc != hipSuccess) {
    (void)hipGraphDestroy(g);
    KPA_HIP(rc);
  }
  kpa_graph_s* h = new (std::nothrow) kpa_graph_s;
  if (!h) {
    (void)hipGraphExecDestroy(e);
    (void)hipGraphDestroy(g);
    KPA_REQUIRE(false, KPA_EINVAL, "out of host memory");
  }
  h->graph = g;
  h->exec = e;
  *out = h;
  return KPA_OK;
}

kpa_status kpa_graph_launch(kpa_graph g, hipStream_t stream) {
  clear_error();
  KPA_REQUIRE(g != nullptr && g->exec != nullptr, KPA_EINVAL, "null graph");
  KPA_HIP(hipGraphLaunch(g->exec, stream));
  return KPA_OK;
}

kpa_status kpa_graph_destroy(kpa_graph g) {
  clear_error();
  if (!g) return KPA_OK;
  hipError_t a = g->exec ? hipGraphExecDestroy(g->exec) : hipSuccess;
  hipError_t b = g->graph ? hipGraphDestroy(g->graph) : hipSuccess;
  delete g;
  KPA_HIP(a);
  KPA_HIP(b);
  return KPA_OK;
}

}  // extern "C"
