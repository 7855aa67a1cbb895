// Pippenger's bucket method for sum_j s_j P_j over G1 and G2 (Groth16's
// A, B, L and H queries), plus fixed-base batch multiplication for key
// generation.
//
// Device pipeline for one MSM with window width c and nw signed windows:
//   1. digits:  each scalar is folded to |s| <= (r-1)/2 with a sign (s > (r-1)/2
//               becomes -(r - s)) and recoded into signed digits in
//               (-2^(c-1), 2^(c-1)]; digit d != 0 of window w names bucket
//               |d| - 1 of that window and carries the sign.  A histogram of
//               bucket sizes is built with atomics.
//   2. sort:    an exclusive scan of the histogram gives each bucket's range;
//               a scatter places (point index | sign) into it (counting sort;
//               the order inside a bucket is irrelevant to the sum).
//   3. accumulate: every bucket is cut into tasks of at most K entries, one
//               thread per task, so work stays balanced whatever the bucket
//               sizes (small-integer scalars pile into few buckets).  Each
//               task sums its points with mixed XYZZ additions.  The partial
//               sums of a bucket are contiguous, so the same cut-and-sum step
//               repeats on them until every bucket holds one point.
//   4. reduce:  per window, sum_b (b+1) B_b by running sums over segments of
//               buckets plus a small multiple of each segment total, then a
//               tree sum over segments.
//   5. host:    sum_w 2^(c w) W_w by Horner's rule (a serial chain of about 254
//               doublings, which one CPU core does far faster than one wave).
#include "msm.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "curve.hpp"
#include "field.hpp"
#include "profile.hpp"
#include "scan.hpp"

namespace zkvc {

constexpr uint32_t EMPTY = 0xffffffffu;
constexpr uint32_t WG_TASK_ENTRIES = 256;  // entries per large-bucket (wavefront) task
constexpr uint32_t SIGN = 0x80000000u;
enum MsmSlot {
  S_DIGITS = 100, S_COUNTS, S_OFFSETS, S_CURSOR, S_SORTED, S_TASKS, S_CNT_A, S_CNT_B, S_OFF_A, S_OFF_B,
  S_PART0, S_PART1, S_SCRATCH, S_SCRATCH2, S_SEG, S_WIN, S_META, S_FB_XYZZ, S_FB_PREFIX, S_UNUSED
};

__device__ __forceinline__ uint32_t bitrev_n(uint32_t a, int bits) {
  return bits == 0 ? 0u : (__builtin_bitreverse32(a) >> (32 - bits));
}

// ---------------------------------------------------------------- 1. digits
struct DigitParams {
  const uint32_t* scalars;
  uint32_t nscalars;
  const uint32_t* points;
  uint32_t npoints;
  int mont, bitrev_bits, c, nw;
  uint32_t nb;
  uint32_t* digits;
  uint32_t* counts;
};

template <class F>
__global__ void k_msm_digits(DigitParams p) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= p.nscalars) return;
  const uint32_t idx = p.bitrev_bits ? bitrev_n(j, p.bitrev_bits) : j;
  bool skip = idx >= p.npoints;
  if (!skip) skip = PointIO<F>::affine_is_zero(p.points + (size_t)idx * PointIO<F>::AFF_WORDS);
  uint32_t s[8];
  {
    const uint4 a = reinterpret_cast<const uint4*>(p.scalars + 8ull * j)[0];
    const uint4 b = reinterpret_cast<const uint4*>(p.scalars + 8ull * j)[1];
    s[0] = a.x; s[1] = a.y; s[2] = a.z; s[3] = a.w; s[4] = b.x; s[5] = b.y; s[6] = b.z; s[7] = b.w;
  }
  if (p.mont) {
    Fr x = Fr::unpack(s);
    x = Fr::from_mont(x);
    x.pack(s);
  }
  // fold: s > (r-1)/2  ->  r - s with the sign flipped
  bool gt = false, decided = false;
#pragma unroll
  for (int k = 7; k >= 0; k--) {
    if (!decided && s[k] != FrParams::HALF32[k]) {
      gt = s[k] > FrParams::HALF32[k];
      decided = true;
    }
  }
  const uint32_t neg = gt ? 1u : 0u;
  if (gt) {
    uint64_t borrow = 0;
#pragma unroll
    for (int k = 0; k < 8; k++) {
      const uint64_t t = (uint64_t)FrParams::P32[k] - s[k] - borrow;
      s[k] = (uint32_t)t;
      borrow = (t >> 32) & 1u;
    }
  }
  const uint32_t half = 1u << (p.c - 1);
  const uint32_t cmask = (1u << p.c) - 1u;
  uint32_t carry = 0;
  for (int w = 0; w < p.nw; w++) {
    const int pos = p.c * w;
    const int q = pos >> 5, sh = pos & 31;
    uint32_t raw = 0;
    if (q < 8) {
      const uint32_t lo = s[q];
      const uint32_t hi = q + 1 < 8 ? s[q + 1] : 0u;
      raw = (uint32_t)((((uint64_t)hi << 32) | lo) >> sh) & cmask;
    }
    uint32_t d = raw + carry;
    uint32_t sgn = 0;
    if (d > half) {
      d = (1u << p.c) - d;
      sgn = 1;
      carry = 1;
    } else {
      carry = 0;
    }
    uint32_t out = EMPTY;
    if (!skip && d != 0u) {
      const uint32_t bucket = d - 1u;
      out = bucket | ((neg ^ sgn) << 31);
      atomicAdd(&p.counts[(size_t)w * p.nb + bucket], 1u);
    }
    p.digits[(size_t)w * p.nscalars + j] = out;
  }
}

// ---------------------------------------------------------------- 2. scatter
__global__ void k_msm_scatter(const uint32_t* digits, uint32_t nscalars, int nw, uint32_t nb, uint32_t* cursor,
                              uint32_t* sorted, int bitrev_bits) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nscalars) return;
  const uint32_t idx = bitrev_bits ? bitrev_n(j, bitrev_bits) : j;
  for (int w = 0; w < nw; w++) {
    const uint32_t d = digits[(size_t)w * nscalars + j];
    if (d == EMPTY) continue;
    const uint32_t b = d & ~SIGN;
    const uint32_t pos = atomicAdd(&cursor[(size_t)w * nb + b], 1u);
    sorted[pos] = idx | (d & SIGN);
  }
}

// ---------------------------------------------------------------- 3. tasks and accumulation
// Buckets are split into tasks by their actual size: a bucket with fewer than
// `large` entries becomes thread tasks of at most K entries (one thread sums a
// task serially); a larger one becomes wavefront tasks of WG_TASK_ENTRIES
// entries reduced by an LDS tree.  nt[f] is the number of partial sums of
// bucket f; a bucket's partial sums are contiguous.
__global__ void k_msm_task_counts(const uint32_t* cnt, uint32_t nbt, uint32_t K, uint32_t large, uint32_t* nt) {
  const uint32_t f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nbt) return;
  const uint32_t c = cnt[f];
  const uint32_t sz = c >= large ? WG_TASK_ENTRIES : K;
  nt[f] = (c + sz - 1) / sz;
}

// Task records (first entry, length, output partial slot); the two task lists
// are filled through atomic counters (their order does not matter).
__global__ void k_msm_make_tasks(const uint32_t* cnt, const uint32_t* off, const uint32_t* part_off, uint32_t nbt,
                                 uint32_t K, uint32_t large, uint32_t* counters, uint4* th_tasks, uint4* wg_tasks) {
  const uint32_t f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nbt) return;
  const uint32_t c = cnt[f];
  if (c == 0) return;
  const uint32_t o = off[f], p = part_off[f];
  const bool big = c >= large;
  const uint32_t sz = big ? WG_TASK_ENTRIES : K;
  const uint32_t nt = (c + sz - 1) / sz;
  const uint32_t base = atomicAdd(&counters[big ? 1 : 0], nt);
  uint4* dst = big ? wg_tasks : th_tasks;
  for (uint32_t q = 0; q < nt; q++) {
    const uint32_t len = c - q * sz < sz ? c - q * sz : sz;
    dst[base + q] = make_uint4(o + q * sz, len, p + q, 0u);
  }
}

template <class F>
__global__ void __launch_bounds__(64) k_msm_acc_points(const uint4* tasks, const uint32_t* d_ntasks, const uint32_t* sorted,
                                 const uint32_t* points, uint32_t* partials) {
  const uint32_t ntasks = *d_ntasks;
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < ntasks; t += gridDim.x * blockDim.x) {
    const uint4 task = tasks[t];
    Xyzz<F> acc = Xyzz<F>::inf();
    for (uint32_t e = task.x; e < task.x + task.y; e++) {
      const uint32_t ref = sorted[e];
      Affine<F> pt = PointIO<F>::load_affine(points + (size_t)(ref & ~SIGN) * PointIO<F>::AFF_WORDS);
      if (ref & SIGN) pt.y = F::neg(pt.y);
      acc = Xyzz<F>::madd(acc, pt);
    }
    PointIO<F>::store_xyzz(partials + (size_t)task.z * PointIO<F>::XYZZ_WORDS, acc);
  }
}

constexpr int WG_THREADS = 64;   // one wavefront per large-bucket task (at most 4 entries per thread)
constexpr int BP_THREADS = 256;  // bit-plane reduction block

// One wavefront per task of up to WG_TASK_ENTRIES entries of one large
// bucket: each lane sums its entries, then an LDS tree reduces the task.
template <class F>
__global__ void __launch_bounds__(WG_THREADS) k_msm_acc_points_wg(const uint4* tasks, const uint32_t* d_ntasks,
                                                                  const uint32_t* sorted, const uint32_t* points,
                                                                  uint32_t* partials) {
  constexpr int XW = PointIO<F>::XYZZ_WORDS;
  __shared__ uint32_t sh[WG_THREADS / 2 * XW];
  const uint32_t ntasks = *d_ntasks;  // uniform: every block runs the same loop count
  for (uint32_t t = blockIdx.x; t < ntasks; t += gridDim.x) {
    const uint4 task = tasks[t];
    Xyzz<F> acc = Xyzz<F>::inf();
    for (uint32_t e = threadIdx.x; e < task.y; e += WG_THREADS) {
      const uint32_t ref = sorted[task.x + e];
      Affine<F> pt = PointIO<F>::load_affine(points + (size_t)(ref & ~SIGN) * PointIO<F>::AFF_WORDS);
      if (ref & SIGN) pt.y = F::neg(pt.y);
      acc = Xyzz<F>::madd(acc, pt);
    }
    for (int o = WG_THREADS / 2; o >= 1; o >>= 1) {
      if ((int)threadIdx.x >= o && (int)threadIdx.x < 2 * o) PointIO<F>::store_xyzz(sh + (threadIdx.x - o) * XW, acc);
      __syncthreads();
      if ((int)threadIdx.x < o) acc = Xyzz<F>::add(acc, PointIO<F>::load_xyzz(sh + threadIdx.x * XW));
      __syncthreads();
    }
    if (threadIdx.x == 0) PointIO<F>::store_xyzz(partials + (size_t)task.z * XW, acc);
  }
}

// Bucket sums: the remaining partials of each bucket, summed in order.
template <class F>
__global__ void __launch_bounds__(64) k_msm_finalize(const uint32_t* cnt, const uint32_t* off, const uint32_t* partials,
                                                     uint32_t nbt, uint32_t* buckets) {
  constexpr int XW = PointIO<F>::XYZZ_WORDS;
  const uint32_t f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nbt) return;
  const uint32_t c = cnt[f], o = off[f];
  Xyzz<F> acc = Xyzz<F>::inf();
  for (uint32_t e = 0; e < c; e++) acc = Xyzz<F>::add(acc, PointIO<F>::load_xyzz(partials + (size_t)(o + e) * XW));
  PointIO<F>::store_xyzz(buckets + (size_t)f * XW, acc);
}

// Bit planes of the bucket reduction: for window w and bit j,
//   S[w c + j] = sum of B_b over the buckets whose digit value b + 1 has bit j set,
// so that window w contributes sum_j 2^j S[w c + j] = sum_b (b + 1) B_b.
// One block per (w, j); each thread sums a strided share, then an LDS tree.
template <class F>
__global__ void __launch_bounds__(BP_THREADS) k_msm_bitplanes(const uint32_t* buckets, uint32_t nb, int c,
                                                              uint32_t* S) {
  constexpr int XW = PointIO<F>::XYZZ_WORDS;
  __shared__ uint32_t sh[BP_THREADS / 2 * XW];
  const uint32_t w = blockIdx.x / c, j = blockIdx.x % c;
  // digit values v in [1, nb] with bit j set: v = ((t >> j) << (j + 1)) | 2^j | (t & (2^j - 1))
  const uint32_t jmask = (1u << j) - 1u;
  const uint32_t count = (j + 1 < (uint32_t)c) ? nb / 2 : 1u;  // bit c-1 is set only in v = nb
  Xyzz<F> acc = Xyzz<F>::inf();
  for (uint32_t t = threadIdx.x; t < count; t += BP_THREADS) {
    const uint32_t v = ((t >> j) << (j + 1)) | (1u << j) | (t & jmask);
    if (v > nb) continue;
    acc = Xyzz<F>::add(acc, PointIO<F>::load_xyzz(buckets + ((size_t)w * nb + v - 1) * XW));
  }
  for (int o = BP_THREADS / 2; o >= 1; o >>= 1) {
    if ((int)threadIdx.x >= o && (int)threadIdx.x < 2 * o) PointIO<F>::store_xyzz(sh + (threadIdx.x - o) * XW, acc);
    __syncthreads();
    if ((int)threadIdx.x < o) acc = Xyzz<F>::add(acc, PointIO<F>::load_xyzz(sh + threadIdx.x * XW));
    __syncthreads();
  }
  if (threadIdx.x == 0) PointIO<F>::store_xyzz(S + (size_t)blockIdx.x * XW, acc);
}

// ---------------------------------------------------------------- host driver
void msm_choose_window(size_t n, int bits, int* c_out, int* nw_out) {
  if (bits < 1) bits = 1;
  double best = 1e300;
  int bc = 1, bnw = bits + 1;
  for (int c = 2; c <= 18; c++) {
    const int nw = (bits + 1 + c - 1) / c;
    // entries + about three group additions per bucket for the reduction
    const double cost = (double)n * nw + 3.0 * nw * (double)(1u << (c - 1));
    if (cost < best) {
      best = cost;
      bc = c;
      bnw = nw;
    }
  }
  *c_out = bc;
  *nw_out = bnw;
}

template <class F>
struct HostOf;
template <>
struct HostOf<Fq> {
  using Pt = host::G1J;
  static host::HFq coord(const uint32_t* w) { return host::HFq::from_dev(w); }
};
template <>
struct HostOf<Fq2> {
  using Pt = host::G2J;
  static host::HFq2 coord(const uint32_t* w) { return hfq2_from_dev(w); }
};

host::HFq2 hfq2_from_dev(const uint32_t* w) { return {host::HFq::from_dev(w), host::HFq::from_dev(w + 8)}; }
void hfq2_to_dev(const host::HFq2& a, uint32_t* w) {
  a.c0.to_dev(w);
  a.c1.to_dev(w + 8);
}

// Sizes of one MSM, all known on the host before any launch, so the device
// pipeline needs no host synchronization until the window sums come back.
struct MsmPlan {
  uint32_t n = 0;
  int c = 0, nw = 0;
  uint32_t nb = 0, nbt = 0;
  uint64_t max_entries = 0;
  uint32_t K = 0;      // entries per thread task
  uint32_t large = 0;  // buckets with at least this many entries get wavefront tasks
  uint64_t max_th_tasks = 0, max_wg_tasks = 0, max_partials = 0;
};

static MsmPlan msm_plan(const MsmInput& in) {
  MsmPlan p;
  p.n = (uint32_t)in.nscalars;
  msm_choose_window(p.n, in.max_bits, &p.c, &p.nw);
  p.nb = 1u << (p.c - 1);
  p.nbt = (uint32_t)p.nw * p.nb;
  p.max_entries = (uint64_t)p.n * p.nw;
  // thread tasks: enough of them to fill the device, long enough to amortize
  p.K = (uint32_t)std::max<uint64_t>(4, std::min<uint64_t>(p.max_entries / 65536, 64));
  p.large = std::max<uint32_t>(64, 8 * p.K);
  p.max_th_tasks = p.max_entries / p.K + p.nbt;
  // a large bucket of c entries makes ceil(c / WG_TASK_ENTRIES) tasks, and at
  // most max_entries / large buckets are large
  p.max_wg_tasks = p.max_entries / WG_TASK_ENTRIES + p.max_entries / p.large + 1;
  p.max_partials = p.max_th_tasks + p.max_wg_tasks;
  return p;
}

template <class F>
void msm_enqueue(const MsmInput& in, Workspace& ws, hipStream_t st, MsmPending& pend) {
  constexpr int XW = PointIO<F>::XYZZ_WORDS;
  ZK_REQUIRE(in.nscalars < (1ull << 31) && in.npoints < (1ull << 31), "MSM too large");
  pend = MsmPending();
  pend.xyzz_words = XW;
  if (in.nscalars == 0) return;
  const MsmPlan p = msm_plan(in);
  ZK_REQUIRE(p.max_entries < (1ull << 32), "MSM too large for 32-bit bucket offsets");
  pend.empty = false;
  pend.c = p.c;
  pend.nw = p.nw;
  const uint32_t n = p.n, nbt = p.nbt;
  const bool g1 = PointIO<F>::AFF_WORDS == 16;

  // all buffers first (growing a buffer synchronizes the device)
  uint32_t* digits = ws.get(S_DIGITS, (size_t)p.nw * n * 4);
  uint32_t* counts = ws.get(S_COUNTS, (size_t)nbt * 4);
  uint32_t* offsets = ws.get(S_OFFSETS, (size_t)nbt * 4);
  uint32_t* cursor = ws.get(S_CURSOR, (size_t)nbt * 4);
  uint32_t* nt = ws.get(S_CNT_A, (size_t)nbt * 4);
  uint32_t* part_off = ws.get(S_OFF_A, (size_t)nbt * 4);
  uint32_t* sorted = ws.get(S_SORTED, p.max_entries * 4);
  uint4* th_tasks = ws.get<uint4>(S_TASKS, p.max_th_tasks * 16);
  uint4* wg_tasks = ws.get<uint4>(S_PART1, p.max_wg_tasks * 16);
  uint32_t* part = ws.get(S_PART0, p.max_partials * XW * 4);
  uint32_t* buckets = ws.get(S_SEG, (size_t)nbt * XW * 4);
  const size_t nplanes = (size_t)p.nw * p.c;
  uint32_t* win = ws.get(S_WIN, nplanes * XW * 4);
  uint32_t* meta = ws.get(S_META, 64 * 4);  // [0] entries [2] partials [8] thread tasks [9] wavefront tasks
  uint32_t* win_host = ws.host<uint32_t>(S_WIN, nplanes * XW * 4);
  ws.get(S_SCRATCH, (size_t)cdiv(nbt, 2048) * 4 + 64);
  pend.win_host = win_host;

  fill_u32(counts, 0u, nbt, st);
  fill_u32(meta + 8, 0u, 2, st);
  DigitParams dp{in.scalars, n, in.points, (uint32_t)in.npoints, in.scalars_mont ? 1 : 0,
                 in.point_index_bitrev, p.c, p.nw, p.nb, digits, counts};
  {
    ProfScope ps(g1 ? "msm_digits_g1" : "msm_digits_g2", st, (double)n);
    hipLaunchKernelGGL(k_msm_digits<F>, dim3(cdiv(n, 256)), dim3(256), 0, st, dp);
    ZK_HIP(hipGetLastError());
  }
  scan_exclusive(counts, offsets, nbt, 0, meta + 0, nullptr, ws, S_SCRATCH, st);
  ZK_HIP(hipMemcpyAsync(cursor, offsets, (size_t)nbt * 4, hipMemcpyDeviceToDevice, st));
  {
    ProfScope ps("msm_scatter", st, (double)n * p.nw);
    hipLaunchKernelGGL(k_msm_scatter, dim3(cdiv(n, 256)), dim3(256), 0, st, digits, n, p.nw, p.nb, cursor, sorted,
                       in.point_index_bitrev);
    ZK_HIP(hipGetLastError());
  }
  // tasks by actual bucket size
  hipLaunchKernelGGL(k_msm_task_counts, dim3(cdiv(nbt, 256)), dim3(256), 0, st, counts, nbt, p.K, p.large, nt);
  ZK_HIP(hipGetLastError());
  scan_exclusive(nt, part_off, nbt, 0, meta + 2, nullptr, ws, S_SCRATCH, st);
  hipLaunchKernelGGL(k_msm_make_tasks, dim3(cdiv(nbt, 256)), dim3(256), 0, st, counts, offsets, part_off, nbt, p.K,
                     p.large, meta + 8, th_tasks, wg_tasks);
  ZK_HIP(hipGetLastError());
  {
    ProfScope ps(g1 ? "msm_acc_points_g1" : "msm_acc_points_g2", st, -1.0);
    // capped grids with stride loops: the task counts are only known on the device
    const unsigned th_grid = (unsigned)std::min<uint64_t>(cdiv(p.max_th_tasks, 64), 65536);
    const unsigned wg_grid = (unsigned)std::min<uint64_t>(p.max_wg_tasks, 8192);
    hipLaunchKernelGGL(k_msm_acc_points<F>, dim3(th_grid), dim3(64), 0, st, th_tasks, meta + 8, sorted, in.points,
                       part);
    ZK_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_msm_acc_points_wg<F>, dim3(wg_grid), dim3(WG_THREADS), 0, st, wg_tasks, meta + 9, sorted,
                       in.points, part);
    ZK_HIP(hipGetLastError());
    ps.set_work_from_device(meta + 0);
  }
  const uint32_t* cur_cnt = nt;
  const uint32_t* cur_off = part_off;
  const uint32_t* cur_part = part;
  {
    ProfScope ps(g1 ? "msm_finalize_g1" : "msm_finalize_g2", st, (double)nbt);
    hipLaunchKernelGGL(k_msm_finalize<F>, dim3(cdiv(nbt, 64)), dim3(64), 0, st, cur_cnt, cur_off, cur_part, nbt,
                       buckets);
    ZK_HIP(hipGetLastError());
  }
  {
    ProfScope ps(g1 ? "msm_bitplanes_g1" : "msm_bitplanes_g2", st, (double)nplanes * p.nb / 2);
    hipLaunchKernelGGL(k_msm_bitplanes<F>, dim3((unsigned)nplanes), dim3(BP_THREADS), 0, st, buckets, p.nb, p.c, win);
    ZK_HIP(hipGetLastError());
  }
  ZK_HIP(hipMemcpyAsync(win_host, win, nplanes * XW * 4, hipMemcpyDeviceToHost, st));
}

// Horner over the windows on the host; call after the MSM's stream has completed.
template <class F>
typename HostOf<F>::Pt msm_finish(const MsmPending& pend) {
  using HP = typename HostOf<F>::Pt;
  constexpr int XW = PointIO<F>::XYZZ_WORDS;
  constexpr int CW = XW / 4;
  HP acc = HP::inf();
  if (pend.empty) return acc;
  // the plane sum of bit position q = c w + j carries weight 2^q
  const int nplanes = pend.nw * pend.c;
  bool started = false;
  for (int q = nplanes - 1; q >= 0; q--) {
    if (started) acc = HP::dbl(acc);
    const uint32_t* e = pend.win_host + (size_t)q * XW;
    bool zero = true;
    for (int k = 2 * CW; k < 3 * CW; k++) zero = zero && e[k] == 0u;  // ZZ = 0: infinity
    if (zero) continue;
    auto X = HostOf<F>::coord(e), Y = HostOf<F>::coord(e + CW), ZZ = HostOf<F>::coord(e + 2 * CW),
         ZZZ = HostOf<F>::coord(e + 3 * CW);
    acc = HP::add(acc, host::xyzz_to_jac(X, Y, ZZ, ZZZ));
    started = true;
  }
  return acc;
}

template <class F>
typename HostOf<F>::Pt msm_run(const MsmInput& in, Workspace& ws, hipStream_t st) {
  MsmPending pend;
  msm_enqueue<F>(in, ws, st, pend);
  ZK_HIP(hipStreamSynchronize(st));
  return msm_finish<F>(pend);
}

void msm_enqueue_g1(const MsmInput& in, Workspace& ws, hipStream_t st, MsmPending& pend) {
  msm_enqueue<Fq>(in, ws, st, pend);
}
void msm_enqueue_g2(const MsmInput& in, Workspace& ws, hipStream_t st, MsmPending& pend) {
  msm_enqueue<Fq2>(in, ws, st, pend);
}
host::G1J msm_finish_g1(const MsmPending& pend) { return msm_finish<Fq>(pend); }
host::G2J msm_finish_g2(const MsmPending& pend) { return msm_finish<Fq2>(pend); }

host::G1J msm_g1(const MsmInput& in, Workspace& ws, hipStream_t st) { return msm_run<Fq>(in, ws, st); }
host::G2J msm_g2(const MsmInput& in, Workspace& ws, hipStream_t st) { return msm_run<Fq2>(in, ws, st); }

// ---------------------------------------------------------------- layout conversion
template <class F>
__global__ void k_points_to_mont(const uint32_t* in, uint32_t* out, uint32_t n) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  constexpr int AW = PointIO<F>::AFF_WORDS;
  Affine<F> a = PointIO<F>::load_affine(in + (size_t)j * AW);
  a.x = F::to_mont(a.x);
  a.y = F::to_mont(a.y);
  PointIO<F>::store_affine(out + (size_t)j * AW, a);
}

void points_to_mont_g1(const uint32_t* in, uint32_t* out, size_t n, hipStream_t st) {
  if (!n) return;
  hipLaunchKernelGGL(k_points_to_mont<Fq>, dim3(cdiv(n, 128)), dim3(128), 0, st, in, out, (uint32_t)n);
  ZK_HIP(hipGetLastError());
}
void points_to_mont_g2(const uint32_t* in, uint32_t* out, size_t n, hipStream_t st) {
  if (!n) return;
  hipLaunchKernelGGL(k_points_to_mont<Fq2>, dim3(cdiv(n, 128)), dim3(128), 0, st, in, out, (uint32_t)n);
  ZK_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- fixed-base batch multiplication
// Table T[w][d] = d * 2^(8w) * G (affine, w < 32, d < 256): [k]G is the sum of
// one table entry per byte of k, i.e. at most 32 mixed additions.
constexpr int FB_WINDOWS = 32;
constexpr int FB_ENTRIES = 256;

template <class F>
__global__ void __launch_bounds__(64) k_fixed_base(const uint32_t* scalars, int mont, uint32_t n, const uint32_t* table, uint32_t* xyzz) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  uint32_t s[8];
  {
    const uint4 a = reinterpret_cast<const uint4*>(scalars + 8ull * j)[0];
    const uint4 b = reinterpret_cast<const uint4*>(scalars + 8ull * j)[1];
    s[0] = a.x; s[1] = a.y; s[2] = a.z; s[3] = a.w; s[4] = b.x; s[5] = b.y; s[6] = b.z; s[7] = b.w;
  }
  if (mont) {
    Fr x = Fr::unpack(s);
    x = Fr::from_mont(x);
    x.pack(s);
  }
  constexpr int AW = PointIO<F>::AFF_WORDS;
  Xyzz<F> acc = Xyzz<F>::inf();
  for (int w = 0; w < FB_WINDOWS; w++) {
    const uint32_t byte = (s[w >> 2] >> (8 * (w & 3))) & 0xffu;
    if (byte) acc = Xyzz<F>::madd(acc, PointIO<F>::load_affine(table + ((size_t)w * FB_ENTRIES + byte) * AW));
  }
  PointIO<F>::store_xyzz(xyzz + (size_t)j * PointIO<F>::XYZZ_WORDS, acc);
}

// XYZZ -> affine with Montgomery's simultaneous inversion over chunks of CH
// points per thread: 1/ZZZ for every point from one field inversion, then
// y = Y / ZZZ and x = X (ZZ / ZZZ)^2 (since ZZ^3 = ZZZ^2).  Infinity -> (0, 0).
constexpr int BA_CHUNK = 16;

template <class F>
__global__ void __launch_bounds__(64) k_batch_affine(const uint32_t* xyzz, uint32_t n, uint32_t* prefix, uint32_t* out, int canonical) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t j0 = t * BA_CHUNK;
  if (j0 >= n) return;
  const uint32_t j1 = j0 + BA_CHUNK < n ? j0 + BA_CHUNK : n;
  constexpr int XW = PointIO<F>::XYZZ_WORDS;
  constexpr int CW = XW / 4;
  constexpr int AW = PointIO<F>::AFF_WORDS;
  F acc = F::one();
  for (uint32_t j = j0; j < j1; j++) {
    acc.store(prefix + (size_t)j * CW);  // product of the nonzero ZZZ before j
    const F z = F::load(xyzz + (size_t)j * XW + 3 * CW);
    if (!F::is_zero(z)) acc = F::mul(acc, z);
  }
  F inv = F::inv(acc);
  for (uint32_t jj = j1; jj > j0; jj--) {
    const uint32_t j = jj - 1;
    const uint32_t* p = xyzz + (size_t)j * XW;
    const F z = F::load(p + 3 * CW);
    Affine<F> a;
    if (F::is_zero(z)) {
      a.x = F::zero();
      a.y = F::zero();
    } else {
      const F zinv = F::mul(inv, F::load(prefix + (size_t)j * CW));
      inv = F::mul(inv, z);
      const F t2 = F::mul(F::load(p + 2 * CW), zinv);  // ZZ / ZZZ = 1/z
      a.x = F::mul(F::load(p), F::sqr(t2));
      a.y = F::mul(F::load(p + CW), zinv);
      if (canonical) {
        a.x = F::from_mont(a.x);
        a.y = F::from_mont(a.y);
      }
    }
    PointIO<F>::store_affine(out + (size_t)j * AW, a);
  }
}

namespace {

template <class HFt>
void batch_invert_host(std::vector<HFt>& v) {
  std::vector<HFt> pre(v.size());
  HFt acc = HFt::one();
  for (size_t i = 0; i < v.size(); i++) {
    pre[i] = acc;
    acc = HFt::mul(acc, v[i]);
  }
  HFt inv = HFt::inv(acc);
  for (size_t i = v.size(); i-- > 0;) {
    HFt vi = HFt::mul(inv, pre[i]);
    inv = HFt::mul(inv, v[i]);
    v[i] = vi;
  }
}

// Generators in canonical form.
const uint64_t G1X[4] = {1, 0, 0, 0}, G1Y[4] = {2, 0, 0, 0};
void g2_generator(host::HFq2& x, host::HFq2& y) {
  x = {host::HFq::from_u64(G2Gen::X0), host::HFq::from_u64(G2Gen::X1)};
  y = {host::HFq::from_u64(G2Gen::Y0), host::HFq::from_u64(G2Gen::Y1)};
}

template <class HFt>
DevBuf* build_fb_table(const HFt& gx, const HFt& gy, int words_per_coord,
                       void (*to_dev)(const HFt&, uint32_t*)) {
  using J = host::Jac<HFt>;
  const int total = FB_WINDOWS * FB_ENTRIES;
  std::vector<J> pts(total);
  J base = J::from_affine(gx, gy);
  for (int w = 0; w < FB_WINDOWS; w++) {
    pts[w * FB_ENTRIES] = J::inf();
    for (int d = 1; d < FB_ENTRIES; d++) pts[w * FB_ENTRIES + d] = J::add(pts[w * FB_ENTRIES + d - 1], base);
    for (int k = 0; k < 8; k++) base = J::dbl(base);
  }
  // batch affine: x = X/Z^2, y = Y/Z^3
  std::vector<HFt> zs(total);
  for (int i = 0; i < total; i++) zs[i] = pts[i].is_inf() ? HFt::one() : pts[i].Z;
  batch_invert_host(zs);
  std::vector<uint32_t> host((size_t)total * 2 * words_per_coord, 0u);
  for (int i = 0; i < total; i++) {
    if (pts[i].is_inf()) continue;
    HFt zi2 = HFt::sqr(zs[i]);
    HFt x = HFt::mul(pts[i].X, zi2);
    HFt y = HFt::mul(pts[i].Y, HFt::mul(zi2, zs[i]));
    to_dev(x, &host[(size_t)i * 2 * words_per_coord]);
    to_dev(y, &host[(size_t)i * 2 * words_per_coord + words_per_coord]);
  }
  auto* b = new DevBuf(host.size() * 4);
  ZK_HIP(hipMemcpy(b->get(), host.data(), host.size() * 4, hipMemcpyHostToDevice));
  return b;
}

void hfq_to_dev(const host::HFq& a, uint32_t* w) { a.to_dev(w); }

const uint32_t* fb_table_g1() {
  static std::mutex mu;
  static std::map<int, DevBuf*> cache;
  std::lock_guard<std::mutex> lock(mu);
  const int dev = current_device();
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second->get();
  DevBuf* b = build_fb_table<host::HFq>(host::HFq::from_u64(G1X), host::HFq::from_u64(G1Y), 8, hfq_to_dev);
  cache[dev] = b;
  return b->get();
}

const uint32_t* fb_table_g2() {
  static std::mutex mu;
  static std::map<int, DevBuf*> cache;
  std::lock_guard<std::mutex> lock(mu);
  const int dev = current_device();
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second->get();
  host::HFq2 x, y;
  g2_generator(x, y);
  DevBuf* b = build_fb_table<host::HFq2>(x, y, 16, hfq2_to_dev);
  cache[dev] = b;
  return b->get();
}

template <class F>
void fixed_base_run(const uint32_t* table, const uint32_t* scalars, bool mont, size_t n, uint32_t* out,
                    bool canonical, Workspace& ws, hipStream_t st) {
  if (!n) return;
  ZK_REQUIRE(n < (1ull << 31), "batch too large");
  constexpr int XW = PointIO<F>::XYZZ_WORDS;
  uint32_t* xyzz = ws.get(S_FB_XYZZ, n * XW * 4);
  uint32_t* prefix = ws.get(S_FB_PREFIX, n * (XW / 4) * 4);
  hipLaunchKernelGGL(k_fixed_base<F>, dim3(cdiv(n, 64)), dim3(64), 0, st, scalars, mont ? 1 : 0, (uint32_t)n, table,
                     xyzz);
  ZK_HIP(hipGetLastError());
  const size_t nthreads = cdiv(n, BA_CHUNK);
  hipLaunchKernelGGL(k_batch_affine<F>, dim3(cdiv(nthreads, 64)), dim3(64), 0, st, xyzz, (uint32_t)n, prefix, out,
                     canonical ? 1 : 0);
  ZK_HIP(hipGetLastError());
}

}  // namespace

void fixed_base_g1(const uint32_t* scalars, bool scalars_mont, size_t n, uint32_t* out, bool out_canonical,
                   Workspace& ws, hipStream_t st) {
  fixed_base_run<Fq>(fb_table_g1(), scalars, scalars_mont, n, out, out_canonical, ws, st);
}
void fixed_base_g2(const uint32_t* scalars, bool scalars_mont, size_t n, uint32_t* out, bool out_canonical,
                   Workspace& ws, hipStream_t st) {
  fixed_base_run<Fq2>(fb_table_g2(), scalars, scalars_mont, n, out, out_canonical, ws, st);
}

}  // namespace zkvc
