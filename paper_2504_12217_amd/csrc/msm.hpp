// Pippenger multi-scalar multiplication over G1 and G2.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "host_field.hpp"
#include "util.hpp"

namespace zkvc {

struct MsmInput {
  const uint32_t* points = nullptr;   // affine, device Montgomery layout, (0,0) = infinity
  size_t npoints = 0;                 // number of valid points
  const uint32_t* scalars = nullptr;  // Fr elements, 8 words each
  size_t nscalars = 0;
  bool scalars_mont = false;          // scalars in device Montgomery form
  int point_index_bitrev = 0;         // if > 0: scalar j pairs with point bitrev_{bits}(j)
  int max_bits = 254;                 // |s| <= 2^max_bits after sign folding (s > (r-1)/2 -> s - r)
  // Precomputed windows: if pre_c > 0, points holds pre_nw arrays of npoints
  // points each (window-major), window w holding 2^(pre_c w) P_i; the MSM then
  // uses that window width and one set of buckets for all windows.
  int pre_c = 0;
  int pre_nw = 0;
  // Use the autotuner's window width and task size where it set one (else
  // the built-in rules, whose workspace size depends on n alone).
  bool use_tuning = true;
};

// An MSM enqueued on a stream; its bit-plane sums land in pinned host memory.
struct MsmPending {
  bool empty = true;
  int c = 0, nw = 0;
  int xyzz_words = 0;
  const uint32_t* win_host = nullptr;
};

// Enqueue one device pipeline for njobs MSMs (any number) over the same
// group, with no host synchronization; the workspace must not be used by
// anything else until the stream completes.  pend[q] receives job q's
// pending result.
// prio = 1 marks a batch on the critical path: its waves take instruction
// issue ahead of concurrent kernels' waves (s_setprio); results are unchanged.
void msm_enqueue_batch_g1(const MsmInput* in, int njobs, Workspace& ws, hipStream_t st, MsmPending* pend,
                          int prio = 0);
void msm_enqueue_batch_g2(const MsmInput* in, int njobs, Workspace& ws, hipStream_t st, MsmPending* pend,
                          int prio = 0);
// Device and host workspace bytes that msm_enqueue_batch_g1/g2 takes for
// these jobs from a workspace in arena mode (each slot once, 256-byte aligned).
void msm_arena_need(const MsmInput* in, int njobs, int group, size_t* dev_bytes, size_t* host_bytes);
// After the stream has completed: combine one job's bit planes (host).
host::G1J msm_finish_g1(const MsmPending& pend);
host::G2J msm_finish_g2(const MsmPending& pend);

// Returns sum_j s_j P_idx(j) as a host Jacobian point (enqueue, wait, finish).  The bulk work (digit
// recoding, counting sort by bucket, bucket accumulation, bit-plane reduction)
// runs on the device; the host combines the plane sums.
host::G1J msm_g1(const MsmInput& in, Workspace& ws, hipStream_t st);
host::G2J msm_g2(const MsmInput& in, Workspace& ws, hipStream_t st);

// Pick the window width c and the number of signed windows for n terms with
// scalars of at most `bits` bits (after folding s > (r-1)/2 to -(r - s)).
void msm_choose_window(size_t n, int bits, int* c, int* nw);
// The same for fixed points with precomputed windows (nw copies of the
// points, at most max_copies); returns nw = 1 when precomputation does not pay.
void msm_choose_precomputed(size_t n, int bits, int max_copies, int* c, int* nw);

// Fixed-base batch multiplication by the standard generator: out_j = [k_j] G,
// written affine (device Montgomery layout unless out_canonical).
void fixed_base_g1(const uint32_t* scalars, bool scalars_mont, size_t n, uint32_t* out, bool out_canonical,
                   Workspace& ws, hipStream_t st);
void fixed_base_g2(const uint32_t* scalars, bool scalars_mont, size_t n, uint32_t* out, bool out_canonical,
                   Workspace& ws, hipStream_t st);

// Canonical <-> internal layout conversion of affine point arrays.
void points_to_mont_g1(const uint32_t* in, uint32_t* out, size_t n, hipStream_t st);
void points_to_mont_g2(const uint32_t* in, uint32_t* out, size_t n, hipStream_t st);

// Host helpers: internal device words <-> host field elements.
host::HFq2 hfq2_from_dev(const uint32_t* w);
void hfq2_to_dev(const host::HFq2& a, uint32_t* w);

}  // namespace zkvc
