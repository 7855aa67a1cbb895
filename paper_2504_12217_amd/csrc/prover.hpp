// Groth16 for the matrix-multiplication circuits: proving key layout and the
// setup / prove drivers.
#pragma once
#include <hip/hip_runtime.h>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <functional>
#include <future>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "host_field.hpp"
#include "util.hpp"
#include "zkvc.h"

namespace zkvc {

// A contiguous range of variables that one proving-key query covers, with a
// bound on the bit length of their values (after folding to a signed view),
// which sets the MSM window.
struct Seg {
  uint64_t var_start = 0;
  uint64_t count = 0;
  int bits = 253;             // |value| <= 2^bits after sign folding
  uint64_t index = 0;         // first query index of this range (segments are consecutive)
  uint64_t point_offset = 0;  // first stored point of this range inside the query array
  // Precomputed windows: the range is stored pre_nw times, copy w holding
  // 2^(pre_c w) times each point (pre_nw = 1: stored once, no precomputation).
  int pre_c = 0;
  int pre_nw = 1;
};

// Sizes and variable layout of one circuit (see r1cs_layout()).
struct Layout {
  uint32_t a = 0, n = 0, b = 0, kind = 0;
  uint64_t ell = 0;       // public inputs: a*n + a*b
  uint64_t m = 0;         // multiplication constraints
  uint64_t naux = 0;      // auxiliary witness variables
  uint64_t nv = 0;        // 1 + ell + n*b + naux
  int log_n = 0;          // domain 2^log_n >= m + ell + 1
  uint64_t N = 0;
  uint64_t w_start = 0;   // first W variable (= first witness variable) = ell + 1
  uint64_t aux_start = 0; // first auxiliary variable
  int y_bits = 0, aux_bits = 253;
  std::vector<Seg> segA, segB, segL;  // query coverage
  Seg segH;                            // the H query (the Lagrange basis of the coset g H: N points)
  // CRPC kinds: one base per constraint row k < n (the B1, B2 and L entries
  // of w_k0), stored with precomputed windows; the prover sums the n b
  // W terms of those queries as n row terms (see msm_jobs)
  Seg segR;
};

Layout r1cs_layout(uint32_t a, uint32_t n, uint32_t b, uint32_t kind);
bool kind_uses_z(uint32_t kind);

// Witness generation for one proof (the kernels of the Groth16 prover):
// Y = X W (device int32), the assignment (canonical words, L.nv elements) and
// rows 0 .. rows-1 of the evaluation vectors <A_c,a>, <B_c,a>, <C_c,a>
// (canonical words).  zpow: z^e for e < a b (device Montgomery form) for the
// CRPC kinds.  X and W are device copies.
void enqueue_witness_one(const Layout& L, const uint32_t* zpow, uint64_t rows, const int8_t* X, const int8_t* W,
                         int32_t* Y, uint32_t* assign, uint32_t* aev, uint32_t* bev, uint32_t* cev, Workspace& ws,
                         hipStream_t st);
// Estimated device workspace of one proof of this circuit in a batch: the
// assignment and three evaluation vectors, and its share of the MSM
// pipelines (about 48 bytes per scalar: digits, sorted entries, partial sums).
size_t prove_footprint(const Layout& L);
// out[e] = z^e for e < count (device Montgomery form), z_dev one element in that form.
void enqueue_zpow(const uint32_t* z_dev, uint32_t count, uint32_t* out, hipStream_t st);

}  // namespace zkvc

namespace zkvc {

// Host bookkeeping of a begun batch (defined with the prover).
struct BatchRun;
struct BatchRunDeleter {
  void operator()(BatchRun* r) const;
};
using BatchRunPtr = std::unique_ptr<BatchRun, BatchRunDeleter>;

// The resources of one batch in flight: events, one workspace per MSM lane,
// batch-level tables, and one workspace per proof (witness, evaluation
// vectors, quotient, pinned staging).
struct ProveGen {
  hipEvent_t witness_ev = nullptr;   // assignments complete
  hipEvent_t wrow_ev = nullptr;      // the G2 lane's scalars ready (CRPC row values, or the whole witness)
  hipEvent_t quotient_ev = nullptr;  // every h complete (and the tail flag copied)
  hipEvent_t done_ev[3] = {};        // each lane's batch complete
  hipEvent_t lane_t[3] = {};         // the same, with timing
  hipEvent_t ev[3] = {};             // stage timing on the calling stream
  hipEvent_t join_ev[3] = {};        // each lane's end, joined into the graph stream (capture)
  hipEvent_t fork_ev = nullptr;      // calling stream -> graph stream
  hipEvent_t graph_ev = nullptr;     // graph stream -> calling stream
  Workspace lane_ws[3];
  Workspace shared;
  std::vector<std::unique_ptr<Workspace>> slot_ws;
  // Graph replay: a batch with the same composition as the previous one on
  // this generation (the same keys in the same order, the same stream and
  // tuning) is captured into a HIP graph; later batches of that composition
  // replay it after restaging their inputs.  Every buffer the graph touches
  // belongs to this generation and keeps its address between batches.
  std::vector<uint64_t> seen_key;    // composition of the last batch begun here
  std::vector<uint64_t> graph_key;   // composition of the captured graph
  hipGraphExec_t graph = nullptr;
  BatchRunPtr graph_run;             // bookkeeping of the captured batch
  std::vector<int> graph_prof;       // profiling slots recorded by the graph
};

// A few persistent host threads for a context's concurrent host work (the
// lane enqueues of a batch's begin, the per-lane combination of its finish),
// so that no thread is created per proof.  Tasks must not wait for each other.
class TaskPool {
 public:
  explicit TaskPool(int nthreads);
  ~TaskPool();
  TaskPool(const TaskPool&) = delete;
  TaskPool& operator=(const TaskPool&) = delete;
  std::future<void> run(std::function<void()> fn);

 private:
  std::vector<std::thread> threads_;
  std::deque<std::packaged_task<void()>> queue_;
  std::mutex mu_;
  std::condition_variable cv_;
  bool stop_ = false;
};

// Device and host state for proving: the three MSM lanes (streams) and two
// generations of per-batch resources, so that a batch can be enqueued while
// the previous one is still on the device (continuous batching).  A proving
// key owns one for its single proofs; the batch entry point keeps one per
// (device, stream); each server has its own.  Not thread-safe: callers
// serialize its use.
struct ProveCtx {
  static constexpr int LANES = 3;
  static constexpr int GENS = 2;
  enum Lane { LANE_H = 0, LANE_G1 = 1, LANE_G2 = 2 };
  ProveCtx();
  ~ProveCtx();
  ProveCtx(const ProveCtx&) = delete;
  ProveCtx& operator=(const ProveCtx&) = delete;
  int device = 0;
  bool graphs = true;  // capture and replay repeated compositions
  // Eager lanes: the device's shared lane streams (see shared_lanes in
  // prover.hip); a capture uses the context's own capture lanes instead.
  hipStream_t lanes[LANES] = {};
  hipStream_t cap_lanes[LANES] = {};   // created on the first capture
  hipStream_t graph_stream = nullptr;  // captures and replays run here, ordered after the calling stream
  std::unique_ptr<TaskPool> pool;      // helper threads (at most three tasks at a time)
  ProveGen gen[GENS];
  zkvc_prove_stats last{};
  // Frees the workspaces' retired buffers; no batch of this context may be in flight.
  void release_retired();
  // Device and pinned host bytes held by the context's workspaces.
  size_t device_bytes() const;
  size_t host_bytes() const;
};

}  // namespace zkvc

// The opaque proving key of the C ABI.
struct zkvc_pk {
  ~zkvc_pk();
  uint64_t id = 0;  // unique per key of the process (never reused)
  zkvc::Layout L;
  int device = 0;
  bool has_z = false;
  zkvc::host::HFr z;
  // Queries in the internal layout (affine, Montgomery); segments concatenated.
  zkvc::DevBuf qA, qB1, qB2, qL, qH;
  zkvc::DevBuf qRB1, qRB2, qRL;  // row bases (CRPC kinds), Layout::segR copies each
  zkvc::DevBuf zpow;  // z^e for e < a*b (CRPC kinds), internal Fr layout
  zkvc::host::G1J alpha1, beta1, delta1;
  zkvc::host::G2J beta2, delta2;
  zkvc::host::FixedBaseTable<zkvc::host::HFq> delta1_table;
  zkvc::host::FixedBaseTable<zkvc::host::HFq2> delta2_table;
  zkvc::Workspace ws;                     // setup scratch
  std::unique_ptr<zkvc::ProveCtx> ctx;    // single proofs (created on first use)
  std::mutex mu;
  zkvc_prove_stats last{};
  size_t key_bytes = 0;
};

namespace zkvc {

// Builds the proving key and the verification-key blob.
zkvc_pk* groth16_setup(const Layout& L, const host::HFr toxic[5], const host::HFr* z, std::vector<uint8_t>& vk,
                       hipStream_t st);

// One proof of a batch: Y = X W for the key's shape; X, W, Y are host arrays.
struct ProveJob {
  const zkvc_pk* pk = nullptr;
  const int8_t* X = nullptr;
  const int8_t* W = nullptr;
  host::HFr r, s;
  int32_t* Y = nullptr;
  zkvc_proof* out = nullptr;
  bool device_io = false;  // X, W and Y are device buffers (no staging, no copies)
};

// Proves every job (keys of any shapes and kinds, repeats allowed) with one
// set of launches per stage: batched quotient transforms per domain size and
// three MSM pipelines shared by all proofs.  Each proof equals its single
// proof bit for bit.
void groth16_prove_batch(ProveCtx& ctx, const ProveJob* jobs, size_t njobs, hipStream_t st);

// The same in two halves: begin enqueues all device work of the batch on
// generation g of the context (no host wait); finish waits for it, combines
// and assembles on the host, and writes the outputs.  A generation must be
// finished before it is begun again; the other one may be in flight.
BatchRunPtr prove_batch_begin(ProveCtx& ctx, int g, const ProveJob* jobs, size_t njobs, hipStream_t st,
                              bool pipelined = true);
void prove_batch_finish(ProveCtx& ctx, BatchRun& run);
// Releases a run; one begun but not finished first waits for its device work.
void prove_batch_abandon(BatchRunPtr& run);

// Process-wide switch for graph capture and replay (off by default); returns
// the previous setting.
int set_graphs(int enable);

// Proves Y = X W (a batch of one on the key's own context).  With device_io,
// X, W and Y are device buffers on the key's device.
void groth16_prove(zkvc_pk* pk, const int8_t* X, const int8_t* W, const host::HFr& r, const host::HFr& s,
                   int32_t* Y, zkvc_proof* out, hipStream_t st, bool device_io = false);

// Host verifier (pairing product) over a parsed key.
int groth16_verify(const uint8_t* vk, size_t vk_len, const int8_t* X, const int32_t* Y, const zkvc_proof* proof);

}  // namespace zkvc
