// Opt-in per-kernel timing with HIP events on the launching stream.
//
// When enabled (zkvc_profile_begin), each instrumented launch records a start
// and a stop event around itself and the algorithmic work it performs (for
// example the number of point additions of a bucket-accumulation launch).
// zkvc_profile_read waits for the events and aggregates by kernel name.
#pragma once
#include <hip/hip_ext.h>
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
  // bind: the scope covers exactly one kernel launched by launch_ev with the
  // events from bind_events (eager streams only; a capture records nodes)
  ProfScope(const char* name, hipStream_t st, double work, bool bind = false);
  ~ProfScope();
  void stop();
  // The scope's start and stop events for the one launch it covers; false
  // (and null events) when it records nothing or records graph nodes.
  bool bind_events(hipEvent_t* start, hipEvent_t* stop);
  // A pinned, device-visible host word that a kernel of this scope writes
  // with the work count (no copy launched); null when this scope records nothing.
  uint32_t* work_word();

 private:
  int slot_ = -1;
  bool graph_ = false;
  bool defer_ = false;  // eager bound scope: the launch records the events
  bool bound_ = false;
  hipStream_t st_;
};

// Launches a kernel with optional events bound to its own dispatch
// (hipExtLaunchKernel): the start event takes the kernel's start time and the
// stop event completes with the kernel, so no separate marker packet (each
// holds the stream's next kernel back by a few microseconds) sits between
// this kernel and the next.  Plain launch when both events are null.
template <class K, class... Args>
void launch_ev(hipEvent_t start, hipEvent_t stop, K kernel, dim3 grid, dim3 block, uint32_t shmem, hipStream_t st,
               Args... args) {
  if (start || stop)
    hipExtLaunchKernelGGL(kernel, grid, block, shmem, st, start, stop, 0u, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, shmem, st, args...);
}

}  // namespace zkvc
