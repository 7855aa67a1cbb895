// Error plumbing, device buffers and scratch workspaces for the library.
#pragma once
#include <hip/hip_runtime.h>
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "zkvc.h"

namespace zkvc {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define ZK_HIP(expr)                                                                          \
  do {                                                                                        \
    hipError_t _e = (expr);                                                                   \
    if (_e != hipSuccess)                                                                     \
      throw ::zkvc::Error(ZKVC_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e));   \
  } while (0)

#define ZK_REQUIRE(cond, msg)                                   \
  do {                                                          \
    if (!(cond)) throw ::zkvc::Error(ZKVC_EINVAL, (msg));       \
  } while (0)

void set_last_error(const std::string& m);
size_t memory_budget_bytes();  // optional cap from ZKVC_MEMORY_BUDGET_MB (0 = none)

// Owning device allocation.
class DevBuf {
 public:
  DevBuf() = default;
  explicit DevBuf(size_t bytes) { alloc(bytes); }
  ~DevBuf() { release(); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p_(o.p_), n_(o.n_) { o.p_ = nullptr; o.n_ = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p_ = o.p_; n_ = o.n_; o.p_ = nullptr; o.n_ = 0; }
    return *this;
  }
  void alloc(size_t bytes);
  void release();
  void ensure(size_t bytes) { if (bytes > n_) { release(); alloc(bytes); } }
  template <class T = uint32_t>
  T* get() const { return reinterpret_cast<T*>(p_); }
  size_t size() const { return n_; }

 private:
  void* p_ = nullptr;
  size_t n_ = 0;
};

// Owning pinned host allocation (hipHostMalloc), for asynchronous copies.
class HostBuf {
 public:
  HostBuf() = default;
  ~HostBuf() { release(); }
  HostBuf(const HostBuf&) = delete;
  HostBuf& operator=(const HostBuf&) = delete;
  HostBuf(HostBuf&& o) noexcept : p_(o.p_), n_(o.n_) { o.p_ = nullptr; o.n_ = 0; }
  size_t size() const { return n_; }
  void ensure(size_t bytes);
  void release();
  template <class T = uint32_t>
  T* get() const { return reinterpret_cast<T*>(p_); }

 private:
  void* p_ = nullptr;
  size_t n_ = 0;
};

// Grow-only named scratch buffers.  Not thread-safe by itself: each owner
// (a proving key's MSM lane, or one stream of the standalone calls) has its own.
class Workspace {
 public:
  // A buffer that has to grow is replaced, and the old one is retired rather
  // than freed at once: work still in flight may read it, and freeing device
  // memory waits for the whole device, stalling every other stream (a
  // latency spike for a server).  Retired buffers are freed by
  // release_retired(), which owners call when none of their work is in
  // flight.  A replacement is at least 1.5 times the old size, so a slot
  // retires O(log) buffers and holds at most 1.5 times its largest request.
  template <class T = uint32_t>
  T* get(int slot, size_t bytes) {
    if (arena_) return reinterpret_cast<T*>(carve(dev_slots_, slot, bytes, arena_dev_, arena_dev_cap_, arena_dev_used_));
    auto& b = bufs_[slot];
    const size_t need = bytes < 256 ? 256 : bytes;
    if (need > b.size()) {
      const size_t grow = b.size() ? std::max(need, b.size() + b.size() / 2) : need;
      if (b.size()) retired_.push_back(std::move(b));
      try {
        b.alloc((grow + 255) & ~(size_t)255);
      } catch (const Error& e) {
        if (e.code != ZKVC_ENOMEM || grow == need) throw;
        b.alloc(need);  // the headroom does not fit: the exact size
      }
    }
    return b.get<T>();
  }
  // Host buffers are pinned allocations that kernels may write directly
  // (false in arena mode, whose host arena is ordinary memory).
  bool host_mapped() const { return !arena_; }
  template <class T = uint32_t>
  T* host(int slot, size_t bytes) {
    if (arena_)
      return reinterpret_cast<T*>(carve(host_slots_, slot, bytes, arena_host_, arena_host_cap_, arena_host_used_));
    auto& b = host_[slot];
    const size_t need = bytes < 256 ? 256 : bytes;
    if (need > b.size()) {
      const size_t grow = b.size() ? std::max(need, b.size() + b.size() / 2) : need;
      if (b.size()) retired_host_.push_back(std::move(b));
      b.ensure((grow + 255) & ~(size_t)255);
    }
    return b.get<T>();
  }
  // device bytes held, retired buffers included
  size_t bytes() const {
    size_t s = 0;
    for (auto& kv : bufs_) s += kv.second.size();
    for (auto& b : retired_) s += b.size();
    return s;
  }
  // pinned host bytes held, retired buffers included
  size_t host_bytes() const {
    size_t s = 0;
    for (auto& kv : host_) s += kv.second.size();
    for (auto& b : retired_host_) s += b.size();
    return s;
  }
  // Frees the retired buffers; the caller guarantees no work in flight uses them.
  void release_retired() {
    retired_.clear();
    retired_host_.clear();
  }
  bool has_retired() const { return !retired_.empty() || !retired_host_.empty(); }
  void clear() {
    bufs_.clear();
    host_.clear();
    retired_.clear();
    retired_host_.clear();
  }

  // Arena mode: get() and host() carve their buffers from caller-owned
  // ranges (device and host memory) instead of allocating, each slot once
  // per arena, 256-byte aligned; a request beyond a range throws ZKVC_EINVAL.
  // With null bases nothing is dereferenced by the workspace itself: the
  // returned pointers are offsets, and the used sizes tell what a sequence
  // of requests needs.  set_arena clears earlier carvings.
  void set_arena(void* dev, size_t dev_bytes, void* host, size_t host_bytes) {
    arena_ = true;
    arena_dev_ = static_cast<char*>(dev);
    arena_host_ = static_cast<char*>(host);
    arena_dev_cap_ = dev_bytes;
    arena_host_cap_ = host_bytes;
    arena_dev_used_ = arena_host_used_ = 0;
    dev_slots_.clear();
    host_slots_.clear();
  }
  size_t arena_dev_used() const { return arena_dev_used_; }
  size_t arena_host_used() const { return arena_host_used_; }

 private:
  struct Carved {
    size_t off, size;
  };
  static char* carve(std::map<int, Carved>& slots, int slot, size_t bytes, char* base, size_t cap, size_t& used) {
    const size_t need = bytes < 256 ? 256 : bytes;
    auto it = slots.find(slot);
    if (it != slots.end() && it->second.size >= need) return base ? base + it->second.off : nullptr;
    const size_t off = (used + 255) & ~(size_t)255;
    if (off > cap || need > cap - off)
      throw Error(ZKVC_EINVAL, "request exceeds the fixed scratch buffer (" + std::to_string(cap) + " bytes)");
    slots[slot] = Carved{off, need};
    used = off + need;
    return base ? base + off : nullptr;
  }
  bool arena_ = false;
  char* arena_dev_ = nullptr;
  char* arena_host_ = nullptr;
  size_t arena_dev_cap_ = 0, arena_host_cap_ = 0, arena_dev_used_ = 0, arena_host_used_ = 0;
  std::map<int, Carved> dev_slots_, host_slots_;

  std::map<int, DevBuf> bufs_;
  std::map<int, HostBuf> host_;
  std::vector<DevBuf> retired_;
  std::vector<HostBuf> retired_host_;
};

// One workspace per (device, stream) for the standalone entry points.
struct StreamWorkspace {
  std::mutex mu;
  Workspace ws;
};
StreamWorkspace& stream_workspace(hipStream_t st);

int current_device();

// Records event e on stream st.  While st is capturing a graph, an event
// record node is added after the stream's captured work instead, so that
// every replay of the graph records e at that point.
hipError_t record_event_nothrow(hipEvent_t e, hipStream_t st);
inline void record_event(hipEvent_t e, hipStream_t st) { ZK_HIP(record_event_nothrow(e, st)); }

inline unsigned cdiv(size_t a, size_t b) { return (unsigned)((a + b - 1) / b); }

// Fill a u32 device array with a value (a kernel, so it is safe inside captured graphs).
void fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t st);

}  // namespace zkvc
