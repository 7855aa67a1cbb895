// Kernel-level profiling records and their C-ABI readout.
#include "profile.hpp"

#include <atomic>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "api_common.hpp"
#include "util.hpp"

namespace zkvc {
namespace {

// Records come from fixed pools (events created once, one pinned word each
// for device-side work counts, written by the kernel itself), so recording
// costs two event records per launch.
constexpr int POOL = 8192;

struct Rec {
  const char* name = nullptr;
  double work = 0;
  bool stopped = false;
  bool work_dev = false;
  bool fixed = false;  // ms already measured (a graph replay's record)
  float ms = 0.f;
};

std::mutex g_mu;
std::atomic<bool> g_on{false};
// the kernel names recorded, comma separated, or null: all (interned for the process)
std::atomic<const char*> g_select{nullptr};
std::set<std::string> g_names;
std::atomic<int> g_next{0};
hipEvent_t g_ev[2 * POOL];
uint32_t* g_words = nullptr;  // pinned, POOL words
bool g_ready = false;
Rec g_recs[POOL];
hipStream_t g_st[POOL];

// slots for scopes captured into graphs (owned by their graph until released)
constexpr int GPOOL = 4096;
hipEvent_t g_gev[2 * GPOOL];
uint32_t* g_gwords = nullptr;  // pinned, GPOOL words
Rec g_grecs[GPOOL];
std::vector<int> g_gfree;
thread_local std::vector<int>* t_sink = nullptr;

int graph_slot_alloc() {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ready || g_gfree.empty()) return -1;
  const int k = g_gfree.back();
  g_gfree.pop_back();
  return k;
}

// name is one of the comma-separated names in sel
bool selected(const char* sel, const char* name) {
  const size_t n = std::strlen(name);
  for (const char* p = sel; *p;) {
    const char* e = std::strchr(p, ',');
    const size_t len = e ? (size_t)(e - p) : std::strlen(p);
    if (len == n && std::strncmp(p, name, n) == 0) return true;
    if (!e) break;
    p = e + 1;
  }
  return false;
}

bool capturing(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return cs == hipStreamCaptureStatusActive;
}

}  // namespace

void set_capture_sink(std::vector<int>* sink) { t_sink = sink; }

void collect_graph_slots(const std::vector<int>& slots) {
  if (!profiling_enabled()) return;
  for (int gk : slots) {
    const Rec& r = g_grecs[gk];
    if (!r.stopped) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, g_gev[2 * gk], g_gev[2 * gk + 1]) != hipSuccess) {
      (void)hipGetLastError();
      continue;
    }
    const int k = g_next.fetch_add(1);
    if (k >= POOL) return;
    g_recs[k] = r;
    g_recs[k].work = r.work_dev ? (double)g_gwords[gk] : r.work;
    g_recs[k].work_dev = false;
    g_recs[k].fixed = true;
    g_recs[k].ms = ms;
  }
}

void release_graph_slots(std::vector<int>& slots) {
  std::lock_guard<std::mutex> lock(g_mu);
  for (int k : slots) g_gfree.push_back(k);
  slots.clear();
}

bool profiling_enabled() { return g_on.load(std::memory_order_relaxed); }

ProfScope::ProfScope(const char* name, hipStream_t st, double work, bool bind) : st_(st) {
  if (!profiling_enabled()) return;
  const char* sel = g_select.load(std::memory_order_acquire);
  if (sel && !selected(sel, name)) return;
  if (capturing(st)) {
    if (!t_sink) return;
    const int k = graph_slot_alloc();
    if (k < 0) return;
    g_grecs[k] = Rec();
    g_grecs[k].name = name;
    g_grecs[k].work = work;
    if (record_event_nothrow(g_gev[2 * k], st) != hipSuccess) {
      (void)hipGetLastError();
      std::vector<int> back{k};
      release_graph_slots(back);
      return;
    }
    t_sink->push_back(k);
    slot_ = k;
    graph_ = true;
    return;
  }
  const int k = g_next.fetch_add(1);
  if (k >= POOL) return;
  g_recs[k].name = name;
  g_recs[k].work = work;
  g_recs[k].stopped = false;
  g_recs[k].work_dev = false;
  g_recs[k].fixed = false;
  g_st[k] = st;
  if (bind) {
    defer_ = true;
  } else if (hipEventRecord(g_ev[2 * k], st) != hipSuccess) {
    return;
  }
  slot_ = k;
}

bool ProfScope::bind_events(hipEvent_t* start, hipEvent_t* stop) {
  *start = *stop = nullptr;
  if (slot_ < 0 || graph_ || !defer_) return false;
  *start = g_ev[2 * slot_];
  *stop = g_ev[2 * slot_ + 1];
  bound_ = true;
  return true;
}

uint32_t* ProfScope::work_word() {
  if (slot_ < 0) return nullptr;
  if (graph_) {
    g_grecs[slot_].work_dev = true;
    return g_gwords + slot_;
  }
  g_recs[slot_].work_dev = true;
  return g_words + slot_;
}

void ProfScope::stop() {
  if (slot_ < 0) return;
  if (graph_) {
    if (record_event_nothrow(g_gev[2 * slot_ + 1], st_) == hipSuccess)
      g_grecs[slot_].stopped = true;
  } else if (defer_) {
    g_recs[slot_].stopped = bound_;  // recorded by the launch it was bound to
  } else if (hipEventRecord(g_ev[2 * slot_ + 1], st_) == hipSuccess) {
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
    if (!g_ready) {
      for (auto& e : g_ev) ZK_HIP(hipEventCreate(&e));
      for (auto& e : g_gev) ZK_HIP(hipEventCreate(&e));
      ZK_HIP(hipHostMalloc(reinterpret_cast<void**>(&g_words), POOL * 4, hipHostMallocDefault));
      ZK_HIP(hipHostMalloc(reinterpret_cast<void**>(&g_gwords), GPOOL * 4, hipHostMallocDefault));
      for (int k = GPOOL - 1; k >= 0; k--) g_gfree.push_back(k);
      g_ready = true;
    }
    ZK_HIP(hipDeviceSynchronize());
    g_next = 0;
    g_on = true;
  });
}

int zkvc_profile_select(const char* kernel) {
  return guarded([&] {
    const size_t len = kernel ? std::strlen(kernel) : 0;
    ZK_REQUIRE(len < 4096, "kernel list too long");
    std::lock_guard<std::mutex> lock(g_mu);
    g_select.store(len ? g_names.insert(std::string(kernel)).first->c_str() : nullptr, std::memory_order_release);
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
      float ms = r.ms;
      if (!r.fixed) ZK_HIP(hipEventElapsedTime(&ms, g_ev[2 * k], g_ev[2 * k + 1]));
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
