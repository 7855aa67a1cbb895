// Library plumbing: error strings, device buffers, per-stream workspaces, fills.
#include "util.hpp"

#include <cstdlib>

namespace zkvc {

static thread_local std::string g_last_error;

void set_last_error(const std::string& m) { g_last_error = m; }
const std::string& last_error() { return g_last_error; }

size_t memory_budget_bytes() {
  static const size_t v = [] {
    const char* s = std::getenv("ZKVC_MEMORY_BUDGET_MB");
    return s ? (size_t)std::strtoull(s, nullptr, 10) << 20 : (size_t)0;
  }();
  return v;
}

static std::mutex g_alloc_mu;
static size_t g_allocated = 0;

void DevBuf::alloc(size_t bytes) {
  const size_t budget = memory_budget_bytes();
  {
    std::lock_guard<std::mutex> lock(g_alloc_mu);
    if (budget && g_allocated + bytes > budget)
      throw Error(ZKVC_ENOMEM, "allocation of " + std::to_string(bytes) + " bytes exceeds ZKVC_MEMORY_BUDGET_MB");
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error(ZKVC_ENOMEM, "hipMalloc(" + std::to_string(bytes) + "): " + hipGetErrorString(e));
  }
  p_ = p;
  n_ = bytes;
  std::lock_guard<std::mutex> lock(g_alloc_mu);
  g_allocated += bytes;
}

void DevBuf::release() {
  if (p_) {
    (void)hipFree(p_);
    std::lock_guard<std::mutex> lock(g_alloc_mu);
    g_allocated -= n_;
  }
  p_ = nullptr;
  n_ = 0;
}

void HostBuf::ensure(size_t bytes) {
  if (bytes <= n_) return;
  release();
  void* p = nullptr;
  hipError_t e = hipHostMalloc(&p, bytes, hipHostMallocDefault);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error(ZKVC_ENOMEM, "hipHostMalloc(" + std::to_string(bytes) + "): " + hipGetErrorString(e));
  }
  p_ = p;
  n_ = bytes;
}

void HostBuf::release() {
  if (p_) (void)hipHostFree(p_);
  p_ = nullptr;
  n_ = 0;
}

int current_device() {
  int d = 0;
  ZK_HIP(hipGetDevice(&d));
  return d;
}

hipError_t record_event_nothrow(hipEvent_t e, hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  unsigned long long id = 0;
  hipGraph_t graph = nullptr;
  const hipGraphNode_t* deps = nullptr;
  size_t ndeps = 0;
  hipError_t r = hipStreamGetCaptureInfo_v2(st, &cs, &id, &graph, &deps, &ndeps);
  if (r != hipSuccess) return r;
  if (cs != hipStreamCaptureStatusActive) return hipEventRecord(e, st);
  hipGraphNode_t node = nullptr;
  r = hipGraphAddEventRecordNode(&node, graph, deps, ndeps, e);
  if (r != hipSuccess) return r;
  return hipStreamUpdateCaptureDependencies(st, &node, 1, hipStreamSetCaptureDependencies);
}

StreamWorkspace& stream_workspace(hipStream_t st) {
  static std::mutex mu;
  static std::map<std::pair<int, hipStream_t>, StreamWorkspace*> m;
  std::lock_guard<std::mutex> lock(mu);
  auto key = std::make_pair(current_device(), st);
  auto it = m.find(key);
  if (it != m.end()) return *it->second;
  auto* w = new StreamWorkspace();
  m[key] = w;
  return *w;
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

void fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_fill_u32, dim3(cdiv(n, 256)), dim3(256), 0, st, p, v, n);
  ZK_HIP(hipGetLastError());
}

}  // namespace zkvc

#include "api_common.hpp"

namespace zkvc {

void require_device_range(const void* p, size_t bytes, const char* name) {
  if (p == nullptr) throw Error(ZKVC_EINVAL, std::string(name) + " is null");
  hipPointerAttribute_t attr;
  hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error(ZKVC_EINVAL, std::string(name) + " is not a device pointer");
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
    throw Error(ZKVC_EINVAL, std::string(name) + " is not device memory");
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  e = hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error(ZKVC_EINVAL, std::string(name) + ": cannot query the allocation range");
  }
  const char* b = static_cast<const char*>(base);
  const char* q = static_cast<const char*>(p);
  if (q < b || (size_t)(q - b) + bytes > size)
    throw Error(ZKVC_EINVAL, std::string(name) + " is smaller than the size the call needs");
  if (((uintptr_t)p & 15u) != 0) throw Error(ZKVC_EINVAL, std::string(name) + " must be 16-byte aligned");
}

}  // namespace zkvc
