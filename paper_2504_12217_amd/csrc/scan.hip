// Exclusive scan: one block for small arrays; otherwise three phases (per-tile
// scans with tile totals, a scan of the totals, then a uniform add).  Used for
// bucket offsets in the MSM's counting sort.
#include "scan.hpp"

namespace zkvc {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

__device__ __forceinline__ uint32_t scan_f(uint32_t x, uint32_t div) { return div ? (x + div - 1u) / div : x; }

// Block-wide exclusive scan of one value per thread; returns the block total.
__device__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* excl, uint32_t* sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[wid] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (int w = 0; w < SCAN_THREADS / 64; w++) {
      const uint32_t t = sh[w];
      sh[w] = acc;
      acc += t;
    }
    sh[SCAN_THREADS / 64] = acc;
  }
  __syncthreads();
  *excl = x - v + sh[wid];
  const uint32_t total = sh[SCAN_THREADS / 64];
  __syncthreads();
  return total;
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_tiles(const uint32_t* in, uint32_t* out, uint32_t n,
                                                             uint32_t div, uint32_t* tile_totals, uint32_t* d_max) {
  __shared__ uint32_t sh[SCAN_THREADS / 64 + 1];
  const uint32_t base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
  uint32_t vals[SCAN_ITEMS];
  uint32_t sum = 0, mx = 0;
#pragma unroll
  for (int q = 0; q < SCAN_ITEMS; q++) {
    const uint32_t i = base + q;
    const uint32_t v = i < n ? scan_f(in[i], div) : 0u;
    vals[q] = sum;
    sum += v;
    mx = v > mx ? v : mx;
  }
  uint32_t excl;
  const uint32_t total = block_exclusive_scan(sum, &excl, sh);
#pragma unroll
  for (int q = 0; q < SCAN_ITEMS; q++) {
    const uint32_t i = base + q;
    if (i < n) out[i] = vals[q] + excl;
  }
  if (threadIdx.x == 0) tile_totals[blockIdx.x] = total;
  if (d_max) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const uint32_t y = __shfl_xor(mx, o, 64);
      mx = y > mx ? y : mx;
    }
    if ((threadIdx.x & 63) == 0) atomicMax(d_max, mx);
  }
}

// Scan the tile totals in place (any count) with one block, writing the grand total.
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_totals(uint32_t* totals, uint32_t ntiles, uint32_t* d_total) {
  __shared__ uint32_t sh[SCAN_THREADS / 64 + 1];
  uint32_t carry = 0;
  for (uint32_t start = 0; start < ntiles; start += SCAN_THREADS) {
    const uint32_t i = start + threadIdx.x;
    const uint32_t v = i < ntiles ? totals[i] : 0u;
    uint32_t excl;
    const uint32_t t = block_exclusive_scan(v, &excl, sh);
    if (i < ntiles) totals[i] = excl + carry;
    carry += t;
  }
  if (threadIdx.x == 0 && d_total) *d_total = carry;
}

__global__ void k_scan_add(uint32_t* out, uint32_t n, const uint32_t* tile_prefix) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += tile_prefix[i / SCAN_TILE];
}

// Small arrays in one launch: one block walks the array in tiles of
// SMALL_THREADS * SMALL_ITEMS values (16-byte loads), carrying the running
// total.
constexpr int SMALL_THREADS = 256;  // a small block finds room on a device busy with other kernels
constexpr int SMALL_ITEMS = 32;
constexpr uint32_t SMALL_SCAN_MAX = 1u << 15;

// Up to two independent scans per launch: block 0 takes the first array,
// block 1 (if launched) the second.  Arrays are 16-byte aligned.
struct SmallScan {
  const uint32_t* in;
  uint32_t* out;
  uint32_t* d_total;
  uint32_t* d_max;
};

__global__ void __launch_bounds__(SMALL_THREADS) k_scan_small(SmallScan s0, SmallScan s1, uint32_t n, uint32_t div) {
  const SmallScan& S = blockIdx.x == 0 ? s0 : s1;
  const uint32_t* in = S.in;
  uint32_t* out = S.out;
  uint32_t* d_total = S.d_total;
  uint32_t* d_max = S.d_max;
  __shared__ uint32_t sh[SMALL_THREADS / 64 + 1];
  __shared__ uint32_t shmax[SMALL_THREADS / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t carry = 0, mx = 0;
  for (uint32_t start = 0; start < n; start += SMALL_THREADS * SMALL_ITEMS) {
    const uint32_t base = start + threadIdx.x * SMALL_ITEMS;
    uint32_t vals[SMALL_ITEMS];
    if (base + SMALL_ITEMS <= n) {
      const uint4* v4 = reinterpret_cast<const uint4*>(in + base);
#pragma unroll
      for (int q = 0; q < SMALL_ITEMS / 4; q++) {
        const uint4 v = v4[q];
        vals[4 * q] = v.x;
        vals[4 * q + 1] = v.y;
        vals[4 * q + 2] = v.z;
        vals[4 * q + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int q = 0; q < SMALL_ITEMS; q++) vals[q] = base + q < n ? in[base + q] : 0u;
    }
    uint32_t sum = 0;
#pragma unroll
    for (int q = 0; q < SMALL_ITEMS; q++) {
      const uint32_t v = scan_f(vals[q], div);
      vals[q] = sum;
      sum += v;
      mx = v > mx ? v : mx;
    }
    // block-wide exclusive scan of the per-thread sums
    uint32_t x = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) sh[wid] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t acc = 0;
      for (int w = 0; w < SMALL_THREADS / 64; w++) {
        const uint32_t t = sh[w];
        sh[w] = acc;
        acc += t;
      }
      sh[SMALL_THREADS / 64] = acc;
    }
    __syncthreads();
    const uint32_t excl = carry + x - sum + sh[wid];
    if (base + SMALL_ITEMS <= n) {
      uint4* o4 = reinterpret_cast<uint4*>(out + base);
#pragma unroll
      for (int q = 0; q < SMALL_ITEMS / 4; q++)
        o4[q] = make_uint4(vals[4 * q] + excl, vals[4 * q + 1] + excl, vals[4 * q + 2] + excl, vals[4 * q + 3] + excl);
    } else {
#pragma unroll
      for (int q = 0; q < SMALL_ITEMS; q++)
        if (base + q < n) out[base + q] = vals[q] + excl;
    }
    carry += sh[SMALL_THREADS / 64];
    __syncthreads();
  }
  if (d_max) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const uint32_t y = __shfl_xor(mx, o, 64);
      mx = y > mx ? y : mx;
    }
    if (lane == 0) shmax[wid] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 1; w < SMALL_THREADS / 64; w++) mx = shmax[w] > mx ? shmax[w] : mx;
      *d_max = mx;
    }
  }
  if (threadIdx.x == 0 && d_total) *d_total = carry;
}

void scan_exclusive(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t div, uint32_t* d_total,
                    uint32_t* d_max, Workspace& ws, int slot, hipStream_t st) {
  if (n == 0) {
    if (d_total) fill_u32(d_total, 0u, 1, st);
    if (d_max) fill_u32(d_max, 0u, 1, st);
    return;
  }
  if (n <= SMALL_SCAN_MAX) {
    const SmallScan s0{in, out, d_total, d_max};
    hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(SMALL_THREADS), 0, st, s0, s0, n, div);
    ZK_HIP(hipGetLastError());
    return;
  }
  const uint32_t ntiles = cdiv(n, SCAN_TILE);
  uint32_t* totals = ws.get(slot, (size_t)ntiles * 4);
  if (d_max) fill_u32(d_max, 0u, 1, st);
  hipLaunchKernelGGL(k_scan_tiles, dim3(ntiles), dim3(SCAN_THREADS), 0, st, in, out, n, div, totals, d_max);
  ZK_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(SCAN_THREADS), 0, st, totals, ntiles, d_total);
  ZK_HIP(hipGetLastError());
  if (ntiles > 1) {
    hipLaunchKernelGGL(k_scan_add, dim3(cdiv(n, 256)), dim3(256), 0, st, out, n, totals);
    ZK_HIP(hipGetLastError());
  }
}

void scan_exclusive2(const uint32_t* in0, uint32_t* out0, uint32_t* d_total0, const uint32_t* in1, uint32_t* out1,
                     uint32_t* d_total1, uint32_t n, Workspace& ws, int slot, hipStream_t st) {
  if (n == 0 || n > SMALL_SCAN_MAX) {
    scan_exclusive(in0, out0, n, 0, d_total0, nullptr, ws, slot, st);
    scan_exclusive(in1, out1, n, 0, d_total1, nullptr, ws, slot, st);
    return;
  }
  const SmallScan s0{in0, out0, d_total0, nullptr}, s1{in1, out1, d_total1, nullptr};
  hipLaunchKernelGGL(k_scan_small, dim3(2), dim3(SMALL_THREADS), 0, st, s0, s1, n, 0u);
  ZK_HIP(hipGetLastError());
}

}  // namespace zkvc
