// Settings picked by the autotuner for this process.  Zero means "use the
// built-in rule"; the kernels' results never depend on these, only their speed.
#pragma once
#include <atomic>
#include <cstdint>

namespace zkvc {

struct Tuning {
  // window width of MSMs with wide scalars and no precomputed windows, by
  // group (0 = G1, 1 = G2) and ceil(log2 n)
  std::atomic<int> msm_c[2][33];
  // log2 of the divisor that sizes thread tasks (K = entries >> this), by
  // floor(log2 entries)
  std::atomic<int> msm_kdiv_log[34];
  // largest sub-transform (bits) per NTT pass, by log2 N
  std::atomic<int> ntt_kmax[29];
};

Tuning& tuning();
// A hash of every entry: changes whenever the table does.
uint64_t tuning_fingerprint();

inline int ceil_log2(uint64_t v) {
  int l = 0;
  while ((1ull << l) < v) l++;
  return l;
}
inline int floor_log2(uint64_t v) {
  int l = 0;
  while (v >> (l + 1)) l++;
  return l;
}

}  // namespace zkvc
