// The autotuner: times candidate settings on synthetic inputs on the device
// and keeps the fastest for this process (window width and task size of the
// MSMs, sub-transform size per NTT pass).  Results are exact whatever the
// setting; only the speed differs.
#include "tune.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "api_common.hpp"
#include "msm.hpp"
#include "ntt.hpp"
#include "util.hpp"

namespace zkvc {

Tuning& tuning() {
  static Tuning t{};  // zero-initialized: every entry "use the built-in rule"
  return t;
}

uint64_t tuning_fingerprint() {
  const Tuning& t = tuning();
  uint64_t h = 1469598103934665603ull;  // FNV-1a over every entry
  auto mix = [&](int v) {
    h ^= (uint64_t)(uint32_t)v;
    h *= 1099511628211ull;
  };
  for (auto& row : t.msm_c)
    for (auto& v : row) mix(v.load());
  for (auto& v : t.msm_kdiv_log) mix(v.load());
  for (auto& v : t.ntt_kmax) mix(v.load());
  return h;
}

namespace {

std::mutex g_tune_mu;  // one tuning run or import at a time

// splitmix64: deterministic synthetic inputs
uint64_t splitmix(uint64_t& x) {
  uint64_t z = (x += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// n scalars below 2^253 < r (8 words each)
std::vector<uint32_t> random_scalars(size_t n, uint64_t seed) {
  std::vector<uint32_t> w(8 * n);
  uint64_t x = seed;
  for (size_t i = 0; i < n; i++) {
    for (int k = 0; k < 4; k++) {
      uint64_t v = splitmix(x);
      if (k == 3) v &= (1ull << 61) - 1;
      w[8 * i + 2 * k] = (uint32_t)v;
      w[8 * i + 2 * k + 1] = (uint32_t)(v >> 32);
    }
  }
  return w;
}

struct Timer {
  hipEvent_t a, b;
  Timer() {
    ZK_HIP(hipEventCreate(&a));
    ZK_HIP(hipEventCreate(&b));
  }
  ~Timer() {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
  }
};

// best of `reps` runs of fn (milliseconds), after one warm-up run
template <class Fn>
float time_best(Fn&& fn, hipStream_t st, int reps) {
  Timer t;
  fn();
  ZK_HIP(hipStreamSynchronize(st));
  float best = 1e30f;
  for (int r = 0; r < reps; r++) {
    ZK_HIP(hipEventRecord(t.a, st));
    fn();
    ZK_HIP(hipEventRecord(t.b, st));
    ZK_HIP(hipEventSynchronize(t.b));
    float ms = 0.f;
    ZK_HIP(hipEventElapsedTime(&ms, t.a, t.b));
    best = std::min(best, ms);
  }
  return best;
}

int tune_msm(int group, int min_log, int max_log, hipStream_t st) {
  int set = 0;
  Workspace ws;
  for (int lg = min_log; lg <= max_log; lg++) {
    const size_t n = 1ull << lg;
    const int aw = group == 0 ? 16 : 32;
    DevBuf pts(n * aw * 4), sc(n * 32), ks(n * 32);
    const std::vector<uint32_t> hs = random_scalars(n, 0x5eed0000ull + lg), hk = random_scalars(n, 0xba5e0000ull + lg);
    ZK_HIP(hipMemcpyAsync(sc.get(), hs.data(), n * 32, hipMemcpyHostToDevice, st));
    ZK_HIP(hipMemcpyAsync(ks.get(), hk.data(), n * 32, hipMemcpyHostToDevice, st));
    if (group == 0)
      fixed_base_g1(ks.get(), false, n, pts.get(), false, ws, st);
    else
      fixed_base_g2(ks.get(), false, n, pts.get(), false, ws, st);
    MsmInput in;
    in.points = pts.get();
    in.npoints = n;
    in.scalars = sc.get();
    in.nscalars = n;
    in.max_bits = 253;
    auto run = [&] {
      MsmPending p;
      if (group == 0)
        msm_enqueue_batch_g1(&in, 1, ws, st, &p);
      else
        msm_enqueue_batch_g2(&in, 1, ws, st, &p);
    };
    // the window width around the cost model's choice
    int c0, nw0;
    msm_choose_window(n, 253, &c0, &nw0);
    std::atomic<int>& slot = tuning().msm_c[group][lg];
    float best = 1e30f;
    int best_c = c0;
    for (int c = std::max(2, c0 - 2); c <= std::min(15, c0 + 2); c++) {
      slot = c;
      const float ms = time_best(run, st, 2);
      if (ms < best) {
        best = ms;
        best_c = c;
      }
    }
    slot = best_c;
    set++;
    // the thread-task size for this many bucket entries
    const uint64_t E = n * (uint64_t)((253 + 1 + best_c - 1) / best_c);
    std::atomic<int>& kslot = tuning().msm_kdiv_log[std::min(33, floor_log2(E))];
    float kbest = 1e30f;
    int kbest_v = 16;
    for (int kd = 14; kd <= 18; kd++) {
      kslot = kd;
      const float ms = time_best(run, st, 2);
      if (ms < kbest) {
        kbest = ms;
        kbest_v = kd;
      }
    }
    kslot = kbest_v;
    set++;
  }
  return set;
}

int tune_ntt(int min_log, int max_log, hipStream_t st) {
  int set = 0;
  for (int lg = min_log; lg <= max_log; lg++) {
    const size_t n = 1ull << lg;
    DevBuf v(n * 32);
    const std::vector<uint32_t> h = random_scalars(n, 0x7700ull + lg);
    ZK_HIP(hipMemcpyAsync(v.get(), h.data(), n * 32, hipMemcpyHostToDevice, st));
    std::atomic<int>& slot = tuning().ntt_kmax[lg];
    NttFuse f;
    float best = 1e30f;
    int best_k = 0;
    for (int k = 6; k <= 10; k++) {
      slot = k;
      const float ms = time_best([&] { ntt_launch(v.get(), lg, false, false, f, st); }, st, 3);
      if (ms < best) {
        best = ms;
        best_k = k;
      }
    }
    slot = best_k;
    set++;
  }
  return set;
}

}  // namespace
}  // namespace zkvc

using namespace zkvc;

int zkvc_autotune(uint32_t what, uint32_t min_log, uint32_t max_log, void* hip_stream) {
  int set = 0;
  const int rc = guarded([&] {
    ZK_REQUIRE((what & ~(ZKVC_TUNE_MSM_G1 | ZKVC_TUNE_MSM_G2 | ZKVC_TUNE_NTT)) == 0, "unknown tuning target");
    ZK_REQUIRE(min_log >= 4 && min_log <= max_log && max_log <= 22, "tuning sizes must satisfy 4 <= min <= max <= 22");
    std::lock_guard<std::mutex> lock(g_tune_mu);
    hipStream_t st = (hipStream_t)hip_stream;
    if (what & ZKVC_TUNE_MSM_G1) set += tune_msm(0, (int)min_log, (int)max_log, st);
    if (what & ZKVC_TUNE_MSM_G2) set += tune_msm(1, (int)min_log, std::min<int>((int)max_log, 18), st);
    if (what & ZKVC_TUNE_NTT) set += tune_ntt((int)min_log, (int)max_log, st);
    ZK_HIP(hipStreamSynchronize(st));
  });
  return rc < 0 ? rc : set;
}

int zkvc_tune_export(char* buf, size_t* len) {
  return guarded([&] {
    ZK_REQUIRE(len != nullptr, "len is null");
    std::ostringstream os;
    Tuning& t = tuning();
    for (int g = 0; g < 2; g++)
      for (int l = 0; l < 33; l++)
        if (t.msm_c[g][l].load()) os << (g ? "msm_g2 " : "msm_g1 ") << l << " " << t.msm_c[g][l].load() << "\n";
    for (int l = 0; l < 34; l++)
      if (t.msm_kdiv_log[l].load()) os << "msm_kdiv " << l << " " << t.msm_kdiv_log[l].load() << "\n";
    for (int l = 0; l < 29; l++)
      if (t.ntt_kmax[l].load()) os << "ntt " << l << " " << t.ntt_kmax[l].load() << "\n";
    const std::string s = os.str();
    if (!buf) {
      *len = s.size() + 1;
      return;
    }
    ZK_REQUIRE(*len >= s.size() + 1, "buffer too small");
    std::memcpy(buf, s.c_str(), s.size() + 1);
    *len = s.size() + 1;
  });
}

int zkvc_tune_import(const char* text) {
  return guarded([&] {
    ZK_REQUIRE(text != nullptr, "text is null");
    std::istringstream is(text);
    std::string key;
    int l = 0, v = 0;
    struct Entry {
      std::atomic<int>* slot;
      int v;
    };
    std::vector<Entry> parsed;
    Tuning& t = tuning();
    while (is >> key) {
      ZK_REQUIRE((bool)(is >> l >> v), "malformed tuning line");
      if (key == "msm_g1" || key == "msm_g2") {
        ZK_REQUIRE(l >= 0 && l <= 32 && (v == 0 || (v >= 2 && v <= 15)), "msm window out of range");
        parsed.push_back({&t.msm_c[key == "msm_g2"][l], v});
      } else if (key == "msm_kdiv") {
        ZK_REQUIRE(l >= 0 && l <= 33 && (v == 0 || (v >= 8 && v <= 24)), "msm task divisor out of range");
        parsed.push_back({&t.msm_kdiv_log[l], v});
      } else if (key == "ntt") {
        ZK_REQUIRE(l >= 0 && l <= 28 && (v == 0 || (v >= 1 && v <= 10)), "ntt pass size out of range");
        parsed.push_back({&t.ntt_kmax[l], v});
      } else {
        throw Error(ZKVC_EINVAL, "unknown tuning key: " + key);
      }
    }
    std::lock_guard<std::mutex> lock(g_tune_mu);
    for (const Entry& e : parsed) *e.slot = e.v;
  });
}
