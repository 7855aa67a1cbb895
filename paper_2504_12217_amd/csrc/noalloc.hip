// G1 multi-scalar multiplication that allocates no memory, for callers that
// cannot allocate (code under HIP graph capture, tight serving loops, hosts
// that forbid device allocation).  Same pipeline and result as zkvc_msm_g1;
// its workspace is carved from a fixed device array, `scratch`, and a fixed
// host array instead of being allocated.
//
// The device array lives in this code object: each GPU the library runs on
// holds its own copy, at its own address, until the process ends.  Host code
// must not pass the array's name to a kernel (on the host the name is a
// stand-in, not a device address): the device address is looked up once per
// device with hipGetSymbolAddress and kept.
#include <array>
#include <cstring>
#include <mutex>

#include "api_common.hpp"
#include "msm.hpp"

using namespace zkvc;

namespace {

// Largest n accepted, and the scratch that the built-in MSM plan needs for
// any n up to it with G1 points in either layout (the window width, task
// size and buffer sizes of the plan depend on n alone when the autotuner's
// settings are not used; the largest need over n <= 2^16 is about 47.1 MiB, at
// n = 65535 with canonical points).
constexpr size_t NOALLOC_MAX_N = 1u << 16;
constexpr size_t SCRATCH_BYTES = 56ull << 20;
constexpr size_t HOST_SCRATCH_BYTES = 256u << 10;  // plane sums and the job table
constexpr int MAX_DEVICES = 64;

}  // namespace

static __device__ __align__(256) uint8_t scratch[SCRATCH_BYTES];

namespace {

alignas(256) uint8_t g_host_scratch[HOST_SCRATCH_BYTES];
std::mutex g_mu;  // the scratch arrays are shared: one call at a time in this process
std::array<void*, MAX_DEVICES> g_scratch_ptr{};

// The device address of this device's copy of `scratch` (looked up on the
// first call on each device, with that device current).
void* scratch_ptr(int dev) {
  ZK_REQUIRE(dev >= 0 && dev < MAX_DEVICES, "device index out of range");
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    ZK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    ZK_REQUIRE(p != nullptr, "no device address for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

int zkvc_msm_g1_noalloc(const void* d_points, const void* d_scalars, size_t n, uint32_t flags, zkvc_g1* out,
                        void* hip_stream) {
  return guarded([&] {
    ZK_REQUIRE(out != nullptr, "out is null");
    ZK_REQUIRE((flags & ~ZKVC_LAYOUT_MONT) == 0, "unknown MSM flag");
    ZK_REQUIRE(n <= NOALLOC_MAX_N, "zkvc_msm_g1_noalloc: n = " + std::to_string(n) +
                                       " exceeds the fixed scratch's limit of 65536 points");
    if (n == 0) {
      std::memset(out, 0, sizeof(*out));
      return;
    }
    require_device_range(d_points, n * 64, "d_points");
    require_device_range(d_scalars, n * 32, "d_scalars");
    hipStream_t st = (hipStream_t)hip_stream;
    MsmInput in;
    in.npoints = n;
    in.scalars = static_cast<const uint32_t*>(d_scalars);
    in.nscalars = n;
    in.scalars_mont = flags & ZKVC_LAYOUT_MONT;
    in.max_bits = 253;
    in.use_tuning = false;
    // the whole need, checked before anything is launched
    size_t need_dev = 0, need_host = 0;
    in.points = static_cast<const uint32_t*>(d_points);
    msm_arena_need(&in, 1, 1, &need_dev, &need_host);
    need_dev += (flags & ZKVC_LAYOUT_MONT) ? 0 : ((n * 64 + 255) & ~(size_t)255) + 256;
    ZK_REQUIRE(need_dev <= SCRATCH_BYTES && need_host <= HOST_SCRATCH_BYTES,
               "zkvc_msm_g1_noalloc: the MSM plan exceeds the fixed scratch");
    std::lock_guard<std::mutex> lock(g_mu);
    Workspace ws;
    ws.set_arena(scratch_ptr(current_device()), SCRATCH_BYTES, g_host_scratch, HOST_SCRATCH_BYTES);
    const uint32_t* pts = static_cast<const uint32_t*>(d_points);
    if (!(flags & ZKVC_LAYOUT_MONT)) {
      uint32_t* conv = ws.get(1, n * 64);
      points_to_mont_g1(pts, conv, n, st);
      pts = conv;
    }
    in.points = pts;
    g1_to_abi(msm_g1(in, ws, st), out);
  });
}

}  // extern "C"
