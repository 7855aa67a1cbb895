// A proving server: requests of any shape arrive one by one, and one worker
// thread proves them in batches as they come (continuous batching).
//
// Each batch is every queued request that fits the batch size and the
// memory budget (admission by estimated device footprint).  A batch is
// enqueued on one generation of the worker's proving context while the
// previous batch is still on the device (the other generation), so
// requests that arrive while a batch runs are admitted as soon as the
// worker is free to enqueue and their device work overlaps the running
// batch.  Results are bit-identical to single proofs: batching only changes
// which launches carry a proof, never its arithmetic.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "api_common.hpp"
#include "prover.hpp"
#include "zkvc.h"

using namespace zkvc;

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t ticket = 0;
  ProveJob job;
  std::vector<int8_t> X, W;  // the server's copies of the inputs
  size_t bytes = 0;          // estimated device footprint
  Clock::time_point t_submit, t_start;
};

size_t footprint(const zkvc_pk* pk) { return prove_footprint(pk->L); }

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

}  // namespace

struct zkvc_server {
  uint32_t max_batch = 64;
  uint64_t budget = 0;
  int device = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::unique_ptr<Request>> queue;
  std::map<uint64_t, zkvc_server_result> results;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread worker;
  std::string fatal;  // set if the worker could not start

  void run();
  void complete(std::vector<std::unique_ptr<Request>>& batch, int status, Clock::time_point t_done);
};

void zkvc_server::complete(std::vector<std::unique_ptr<Request>>& batch, int status, Clock::time_point t_done) {
  std::lock_guard<std::mutex> lock(mu);
  for (auto& r : batch) {
    zkvc_server_result res{};
    res.status = status;
    res.batch_size = (uint32_t)batch.size();
    res.queue_ms = ms_between(r->t_submit, r->t_start);
    res.latency_ms = ms_between(r->t_submit, t_done);
    results[r->ticket] = res;
  }
  batch.clear();
  cv_done.notify_all();
}

void zkvc_server::run() {
  hipStream_t st = nullptr;
  std::unique_ptr<ProveCtx> ctx;
  try {
    ZK_HIP(hipSetDevice(device));
    ZK_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    ctx.reset(new ProveCtx());
    // batches differ from one to the next and two are in flight at once:
    // eager launches keep the generations overlapping on the device
    ctx->graphs = false;
  } catch (const std::exception& e) {
    std::lock_guard<std::mutex> lock(mu);
    fatal = e.what();
    stop = true;
    cv_done.notify_all();
    return;
  }
  BatchRunPtr prev;
  std::vector<std::unique_ptr<Request>> prev_reqs;
  size_t prev_bytes = 0;  // estimated footprint of the batch in flight
  int gen = 0;
  for (;;) {
    std::vector<std::unique_ptr<Request>> take;
    {
      std::unique_lock<std::mutex> lock(mu);
      // with nothing in flight: free the buffers that growth replaced, then
      // sleep until work arrives
      if (!prev && queue.empty() && !stop) {
        lock.unlock();
        ctx->release_retired();
        lock.lock();
      }
      if (!prev) cv_work.wait(lock, [&] { return stop || !queue.empty(); });
      if (!prev && queue.empty() && stop) break;
      // admission by footprint: the new batch and the one still in flight
      // share the budget (submit rejects a job that exceeds it alone, so a
      // job always fits once nothing is in flight)
      size_t bytes = prev ? prev_bytes : 0;
      while (!queue.empty() && take.size() < max_batch) {
        const size_t b = queue.front()->bytes;
        if (budget && bytes + b > budget) break;
        bytes += b;
        take.push_back(std::move(queue.front()));
        queue.pop_front();
      }
    }
    size_t take_bytes = 0;
    for (auto& r : take) take_bytes += r->bytes;
    BatchRunPtr cur;
    if (!take.empty()) {
      const Clock::time_point t = Clock::now();
      std::vector<ProveJob> jobs;
      for (auto& r : take) {
        r->t_start = t;
        jobs.push_back(r->job);
      }
      try {
        cur = prove_batch_begin(*ctx, gen, jobs.data(), jobs.size(), st);
        gen ^= 1;
      } catch (const Error& e) {
        set_last_error(e.what());
        complete(take, e.code, Clock::now());
      } catch (const std::exception& e) {
        set_last_error(e.what());
        complete(take, ZKVC_EDEVICE, Clock::now());
      }
    }
    if (prev) {
      int status = ZKVC_OK;
      try {
        prove_batch_finish(*ctx, *prev);
      } catch (const Error& e) {
        status = e.code;
        prove_batch_abandon(prev);
      } catch (const std::exception&) {
        status = ZKVC_EDEVICE;
        prove_batch_abandon(prev);
      }
      prev.reset();
      complete(prev_reqs, status, Clock::now());
    }
    prev = std::move(cur);
    prev_reqs = std::move(take);
    prev_bytes = prev ? take_bytes : 0;
  }
  ctx.reset();
  if (st) (void)hipStreamDestroy(st);
}

int zkvc_server_create(const zkvc_server_config* cfg, zkvc_server** out) {
  return guarded([&] {
    ZK_REQUIRE(cfg && out, "null argument");
    ZK_REQUIRE(cfg->max_batch >= 1, "max_batch must be at least 1");
    std::unique_ptr<zkvc_server> s(new zkvc_server());
    s->max_batch = cfg->max_batch;
    s->budget = cfg->memory_budget;
    s->device = current_device();
    zkvc_server* raw = s.get();
    s->worker = std::thread([raw] { raw->run(); });
    *out = s.release();
  });
}

int zkvc_server_submit(zkvc_server* srv, const zkvc_prove_job* job, uint64_t* ticket) {
  return guarded([&] {
    ZK_REQUIRE(srv && job && ticket, "null argument");
    ZK_REQUIRE(job->pk && job->X && job->W && job->Y_out && job->proof_out, "null argument in the proof job");
    ZK_REQUIRE(job->pk->device == srv->device, "the proving key lives on another device");
    std::unique_ptr<Request> r(new Request());
    const Layout& L = job->pk->L;
    r->X.assign(job->X, job->X + (size_t)L.a * L.n);
    r->W.assign(job->W, job->W + (size_t)L.n * L.b);
    r->job.pk = job->pk;
    r->job.X = r->X.data();
    r->job.W = r->W.data();
    r->job.r = fr_in(job->r, "r");
    r->job.s = fr_in(job->s, "s");
    r->job.Y = job->Y_out;
    r->job.out = job->proof_out;
    r->bytes = footprint(job->pk);
    if (srv->budget && r->bytes > srv->budget)
      throw Error(ZKVC_ENOMEM, "the job's estimated device footprint (" + std::to_string(r->bytes) +
                                   " bytes) exceeds the server's memory budget");
    r->t_submit = Clock::now();
    std::lock_guard<std::mutex> lock(srv->mu);
    ZK_REQUIRE(!srv->stop, srv->fatal.empty() ? "the server is stopping" : srv->fatal);
    r->ticket = srv->next_ticket++;
    *ticket = r->ticket;
    srv->queue.push_back(std::move(r));
    srv->cv_work.notify_one();
  });
}

int zkvc_server_wait(zkvc_server* srv, uint64_t ticket, zkvc_server_result* result) {
  return guarded([&] {
    ZK_REQUIRE(srv && result, "null argument");
    std::unique_lock<std::mutex> lock(srv->mu);
    ZK_REQUIRE(ticket >= 1 && ticket < srv->next_ticket, "unknown ticket");
    srv->cv_done.wait(lock, [&] { return srv->results.count(ticket) || !srv->fatal.empty(); });
    ZK_REQUIRE(srv->fatal.empty(), srv->fatal);
    *result = srv->results[ticket];
    srv->results.erase(ticket);
  });
}

int zkvc_server_destroy(zkvc_server* srv) {
  return guarded([&] {
    if (!srv) return;
    {
      std::lock_guard<std::mutex> lock(srv->mu);
      srv->stop = true;
      srv->cv_work.notify_all();
    }
    if (srv->worker.joinable()) srv->worker.join();
    delete srv;
  });
}
