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

// Records come from fixed pools (events created once, one pinned word each
// for device-side work counts), so recording costs two event records and at
// most one 4-byte copy per launch.
constexpr int POOL = 8192;

struct Rec {
  const char* name = nullptr;
  double work = 0;
  bool stopped = false;
  bool work_dev = false;
};

std::mutex g_mu;
std::atomic<bool> g_on{false};
std::atomic<int> g_next{0};
hipEvent_t g_ev[2 * POOL];
uint32_t* g_words = nullptr;  // pinned, POOL words
bool g_ready = false;
Rec g_recs[POOL];
hipStream_t g_st[POOL];

}  // namespace

bool profiling_enabled() { return g_on.load(std::memory_order_relaxed); }

ProfScope::ProfScope(const char* name, hipStream_t st, double work) : st_(st) {
  if (!profiling_enabled()) return;
  const int k = g_next.fetch_add(1);
  if (k >= POOL) return;
  g_recs[k].name = name;
  g_recs[k].work = work;
  g_recs[k].stopped = false;
  g_recs[k].work_dev = false;
  g_st[k] = st;
  if (hipEventRecord(g_ev[2 * k], st) != hipSuccess) return;
  slot_ = k;
}

void ProfScope::set_work_from_device(const uint32_t* p) {
  if (slot_ < 0) return;
  if (hipMemcpyAsync(g_words + slot_, p, 4, hipMemcpyDeviceToHost, st_) == hipSuccess) g_recs[slot_].work_dev = true;
}

void ProfScope::stop() {
  if (slot_ < 0) return;
  if (hipEventRecord(g_ev[2 * slot_ + 1], st_) == hipSuccess) g_recs[slot_].stopped = true;
  slot_ = -1;
}

ProfScope::~ProfScope() { stop(); }

}  // namespace zkvc

using namespace zkvc;

extern "C" {

int zkvc_profile_begin(void) {
  return guarded([&] {
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ready) {
      for (auto& e : g_ev) ZK_HIP(hipEventCreate(&e));
      ZK_HIP(hipHostMalloc(reinterpret_cast<void**>(&g_words), POOL * 4, hipHostMallocDefault));
      g_ready = true;
    }
    ZK_HIP(hipDeviceSynchronize());
    g_next = 0;
    g_on = true;
  });
}

int zkvc_profile_read(zkvc_kernel_stat* out, int capacity, int* count) {
  return guarded([&] {
    ZK_REQUIRE(count != nullptr, "count is null");
    std::lock_guard<std::mutex> lock(g_mu);
    g_on = false;
    std::map<std::string, zkvc_kernel_stat> agg;
    const int n = std::min<int>(g_next.load(), POOL);
    if (n > 0) ZK_HIP(hipDeviceSynchronize());
    for (int k = 0; k < n; k++) {
      const Rec& r = g_recs[k];
      if (!r.stopped) continue;
      float ms = 0.f;
      ZK_HIP(hipEventElapsedTime(&ms, g_ev[2 * k], g_ev[2 * k + 1]));
      zkvc_kernel_stat& s = agg[r.name];
      std::strncpy(s.name, r.name, sizeof(s.name) - 1);
      s.launches += 1;
      s.total_ms += ms;
      s.work += r.work_dev ? (double)g_words[k] : r.work;
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
