// Opt-in per-kernel timing with HIP events on the launching stream.
//
// When enabled (zkvc_profile_begin), each instrumented launch records a start
// and a stop event around itself and the algorithmic work it performs (for
// example the number of point additions of a bucket-accumulation launch).
// zkvc_profile_read waits for the events and aggregates by kernel name.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

namespace zkvc {

bool profiling_enabled();

// Inside a stream capture a scope records its two events as event nodes of
// the graph, in slots of a separate pool listed in the capturing thread's
// sink; each replay re-records them, and collect_graph_slots adds that
// replay's records to the open profile once the replay has completed.
void set_capture_sink(std::vector<int>* sink);
void collect_graph_slots(const std::vector<int>& slots);
void release_graph_slots(std::vector<int>& slots);

class ProfScope {
 public:
  ProfScope(const char* name, hipStream_t st, double work);
  ~ProfScope();
  void stop();
  // A pinned, device-visible host word that a kernel of this scope writes
  // with the work count (no copy launched); null when this scope records nothing.
  uint32_t* work_word();

 private:
  int slot_ = -1;
  bool graph_ = false;
  hipStream_t st_;
};

}  // namespace zkvc
