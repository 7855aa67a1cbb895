// Integer-VALU peak microbenchmark: the rate at which the device issues
// 32x32 -> 64-bit multiply-adds (v_mad_u64_u32), the instruction every
// partial product of the field arithmetic compiles to.  The bucket
// accumulation and NTT kernels are bound by this rate, so their roofline
// denominator is measured here rather than assumed.
//
// Every thread runs CHAINS independent dependency chains acc_j <- lo(acc_j) *
// m_j + acc_j (one v_mad_u64_u32 each, the 64-bit addend being the previous
// value), so each wave has CHAINS instructions in flight and a compute unit
// holds several waves per SIMD.  Thread 0 of each block also reads the shader
// clock counter (s_memtime) and the constant 100 MHz counter (s_memrealtime)
// around its loop, which gives the clock the device ran at.
#include <cstring>

#include "api_common.hpp"

using namespace zkvc;

namespace {

constexpr int CHAINS = 16;
constexpr int PROBE_THREADS = 256;

__global__ void __launch_bounds__(PROBE_THREADS) k_valu_probe(uint32_t iters, uint32_t seed, uint64_t* sink,
                                                              uint64_t* clocks) {
  uint64_t acc[CHAINS];
  uint32_t m[CHAINS];
#pragma unroll
  for (int j = 0; j < CHAINS; j++) {
    acc[j] = (uint64_t)(seed + threadIdx.x * 7u + (uint32_t)j * 131u) * 0x9e3779b9u;
    m[j] = 0x2545f491u + (uint32_t)j * 2u + blockIdx.x;
  }
  uint64_t c0 = 0, r0 = 0;
  if (threadIdx.x == 0) {
    c0 = clock64();
    r0 = wall_clock64();
  }
  for (uint32_t it = 0; it < iters; it++) {
#pragma unroll
    for (int u = 0; u < 4; u++) {
#pragma unroll
      for (int j = 0; j < CHAINS; j++) acc[j] = (uint64_t)(uint32_t)acc[j] * m[j] + acc[j];
    }
  }
  uint64_t x = 0;
#pragma unroll
  for (int j = 0; j < CHAINS; j++) x ^= acc[j];
  sink[(size_t)blockIdx.x * PROBE_THREADS + threadIdx.x] = x;
  if (threadIdx.x == 0) {
    const uint64_t c1 = clock64(), r1 = wall_clock64();
    clocks[2 * blockIdx.x] = c1 - c0;
    clocks[2 * blockIdx.x + 1] = r1 - r0;
  }
}

}  // namespace

extern "C" {

int zkvc_valu_peak(uint32_t iters, zkvc_valu_peak_t* out, void* hip_stream) {
  return guarded([&] {
    ZK_REQUIRE(out != nullptr, "out is null");
    ZK_REQUIRE(iters >= 1 && iters <= (1u << 20), "iters must be in [1, 2^20]");
    hipStream_t st = (hipStream_t)hip_stream;
    const int dev = current_device();
    int cus = 0, wall_khz = 0;
    ZK_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    ZK_HIP(hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev));
    // 8 blocks of 256 threads per compute unit: 8 waves per SIMD
    const uint32_t blocks = (uint32_t)cus * 8u;
    DevBuf sink((size_t)blocks * PROBE_THREADS * 8), clocks((size_t)blocks * 16);
    hipEvent_t e0, e1;
    ZK_HIP(hipEventCreate(&e0));
    ZK_HIP(hipEventCreate(&e1));
    float ms = 0.f;
    hipError_t err = hipSuccess;
    // one launch to warm the clocks, then the timed one
    for (int rep = 0; rep < 2 && err == hipSuccess; rep++) {
      err = hipEventRecord(e0, st);
      if (err == hipSuccess) {
        hipLaunchKernelGGL(k_valu_probe, dim3(blocks), dim3(PROBE_THREADS), 0, st, iters, (uint32_t)rep,
                           sink.get<uint64_t>(), clocks.get<uint64_t>());
        err = hipGetLastError();
      }
      if (err == hipSuccess) err = hipEventRecord(e1, st);
      if (err == hipSuccess) err = hipEventSynchronize(e1);
      if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ZK_HIP(err);
    std::vector<uint64_t> ck((size_t)blocks * 2);
    ZK_HIP(hipMemcpy(ck.data(), clocks.get(), ck.size() * 8, hipMemcpyDeviceToHost));
    double cyc = 0, wall = 0;
    for (uint32_t b = 0; b < blocks; b++) {
      cyc += (double)ck[2 * b];
      wall += (double)ck[2 * b + 1];
    }
    const double mads = (double)blocks * PROBE_THREADS * iters * 4.0 * CHAINS;
    std::memset(out, 0, sizeof(*out));
    out->compute_units = (uint32_t)cus;
    out->mads = mads;
    out->ms = ms;
    out->mad_per_s = mads / (ms * 1e-3);
    // the shader clock over each block's loop, against the constant counter
    out->clock_ghz = wall > 0 && wall_khz > 0 ? cyc / (wall / (wall_khz * 1e3)) / 1e9 : 0.0;
    out->lane_ops_per_cu_clk =
        out->clock_ghz > 0 ? out->mad_per_s / ((double)cus * out->clock_ghz * 1e9) : 0.0;
  });
}

}  // extern "C"
