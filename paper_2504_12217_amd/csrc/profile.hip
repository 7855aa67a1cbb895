// Kernel-level profiling records and their C-ABI readout.
#include "profile.hpp"

#include <atomic>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "api_common.hpp"

namespace zkvc {
namespace {

struct Rec {
  std::string name;
  hipEvent_t a = nullptr, b = nullptr;
  double work = 0;
  bool stopped = false;
};

std::mutex g_mu;
std::atomic<bool> g_on{false};
std::vector<Rec> g_recs;

}  // namespace

bool profiling_enabled() { return g_on.load(std::memory_order_relaxed); }

ProfScope::ProfScope(const char* name, hipStream_t st, double work) : st_(st) {
  if (!profiling_enabled()) return;
  Rec r;
  r.name = name;
  r.work = work;
  if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) return;
  if (hipEventRecord(r.a, st) != hipSuccess) return;
  std::lock_guard<std::mutex> lock(g_mu);
  g_recs.push_back(r);
  slot_ = (int)g_recs.size() - 1;
}

void ProfScope::stop() {
  if (slot_ < 0) return;
  std::lock_guard<std::mutex> lock(g_mu);
  if (slot_ < (int)g_recs.size() && !g_recs[slot_].stopped) {
    (void)hipEventRecord(g_recs[slot_].b, st_);
    g_recs[slot_].stopped = true;
  }
  slot_ = -1;
}

ProfScope::~ProfScope() { stop(); }

}  // namespace zkvc

using namespace zkvc;

extern "C" {

int zkvc_profile_begin(void) {
  return guarded([&] {
    std::lock_guard<std::mutex> lock(g_mu);
    for (auto& r : g_recs) {
      if (r.a) (void)hipEventDestroy(r.a);
      if (r.b) (void)hipEventDestroy(r.b);
    }
    g_recs.clear();
    g_on = true;
  });
}

int zkvc_profile_read(zkvc_kernel_stat* out, int capacity, int* count) {
  return guarded([&] {
    ZK_REQUIRE(count != nullptr, "count is null");
    std::lock_guard<std::mutex> lock(g_mu);
    g_on = false;
    std::map<std::string, zkvc_kernel_stat> agg;
    for (auto& r : g_recs) {
      if (!r.stopped) continue;
      ZK_HIP(hipEventSynchronize(r.b));
      float ms = 0.f;
      ZK_HIP(hipEventElapsedTime(&ms, r.a, r.b));
      zkvc_kernel_stat& s = agg[r.name];
      std::strncpy(s.name, r.name.c_str(), sizeof(s.name) - 1);
      s.launches += 1;
      s.total_ms += ms;
      s.work += r.work;
    }
    int k = 0;
    for (auto& kv : agg) {
      if (out && k < capacity) out[k] = kv.second;
      k++;
    }
    *count = k;
  });
}

}  // extern "C"
