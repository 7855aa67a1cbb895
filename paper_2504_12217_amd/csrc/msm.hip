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
#include <cstring>
#include <mutex>
#include <vector>

#include "curve.hpp"
#include "field.hpp"
#include "profile.hpp"
#include "scan.hpp"

namespace zkvc {

constexpr uint32_t EMPTY = 0xffffffffu;
constexpr uint32_t SIGN = 0x80000000u;
enum MsmSlot {
  S_DIGITS = 100, S_COUNTS, S_OFFSETS, S_CURSOR, S_SORTED, S_TASKS, S_CNT_A, S_CNT_B, S_OFF_A, S_OFF_B,
  S_PART0, S_PART1, S_SCRATCH, S_SCRATCH2, S_SEG, S_WIN, S_META, S_FB_XYZZ, S_FB_PREFIX
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
__global__ void k_msm_tasks(const uint32_t* cnt, const uint32_t* off, const uint32_t* task_off, uint32_t nbt,
                            uint32_t K, uint2* tasks) {
  const uint32_t f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nbt) return;
  const uint32_t c = cnt[f];
  if (c == 0) return;
  const uint32_t o = off[f], t0 = task_off[f];
  for (uint32_t q = 0; q * K < c; q++) {
    const uint32_t len = c - q * K < K ? c - q * K : K;
    tasks[t0 + q] = make_uint2(o + q * K, len);
  }
}

template <class F>
__global__ void __launch_bounds__(64) k_msm_acc_points(const uint2* tasks, const uint32_t* d_ntasks, const uint32_t* sorted,
                                 const uint32_t* points, uint32_t* partials) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= *d_ntasks) return;
  const uint2 task = tasks[t];
  Xyzz<F> acc = Xyzz<F>::inf();
  for (uint32_t e = task.x; e < task.x + task.y; e++) {
    const uint32_t ref = sorted[e];
    Affine<F> pt = PointIO<F>::load_affine(points + (size_t)(ref & ~SIGN) * PointIO<F>::AFF_WORDS);
    if (ref & SIGN) pt.y = F::neg(pt.y);
    acc = Xyzz<F>::madd(acc, pt);
  }
  PointIO<F>::store_xyzz(partials + (size_t)t * PointIO<F>::XYZZ_WORDS, acc);
}

template <class F>
__global__ void __launch_bounds__(64) k_msm_acc_partials(const uint2* tasks, const uint32_t* d_ntasks, const uint32_t* in,
                                   uint32_t* out) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= *d_ntasks) return;
  const uint2 task = tasks[t];
  constexpr int XW = PointIO<F>::XYZZ_WORDS;
  Xyzz<F> acc = PointIO<F>::load_xyzz(in + (size_t)task.x * XW);
  for (uint32_t e = task.x + 1; e < task.x + task.y; e++)
    acc = Xyzz<F>::add(acc, PointIO<F>::load_xyzz(in + (size_t)e * XW));
  PointIO<F>::store_xyzz(out + (size_t)t * XW, acc);
}

// ---------------------------------------------------------------- 4. bucket reduction
template <class F>
__global__ void __launch_bounds__(64) k_msm_segments(const uint32_t* cnt, const uint32_t* off, const uint32_t* partials, int nw,
                               uint32_t nb, uint32_t L, uint32_t* seg_out) {
  const uint32_t G = nb / L;
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= (uint32_t)nw * G) return;
  const uint32_t w = tid / G, g = tid % G;
  constexpr int XW = PointIO<F>::XYZZ_WORDS;
  Xyzz<F> acc = Xyzz<F>::inf(), sum = Xyzz<F>::inf();
  for (int q = (int)L - 1; q >= 0; q--) {
    const size_t f = (size_t)w * nb + g * L + (uint32_t)q;
    if (cnt[f]) acc = Xyzz<F>::add(acc, PointIO<F>::load_xyzz(partials + (size_t)off[f] * XW));
    sum = Xyzz<F>::add(sum, acc);
  }
  // buckets g*L .. g*L+L-1 hold digit values g*L+1 .. g*L+L: add (g*L) * total
  if (g) sum = Xyzz<F>::add(sum, Xyzz<F>::mul_small(acc, g * L));
  PointIO<F>::store_xyzz(seg_out + (size_t)tid * XW, sum);
}

constexpr int WR_THREADS = 64;

template <class F>
__global__ void __launch_bounds__(WR_THREADS) k_msm_window_reduce(const uint32_t* seg, uint32_t G, uint32_t* win) {
  constexpr int XW = PointIO<F>::XYZZ_WORDS;
  __shared__ uint32_t sh[WR_THREADS * XW];
  const uint32_t w = blockIdx.x;
  Xyzz<F> acc = Xyzz<F>::inf();
  for (uint32_t g = threadIdx.x; g < G; g += WR_THREADS)
    acc = Xyzz<F>::add(acc, PointIO<F>::load_xyzz(seg + ((size_t)w * G + g) * XW));
  for (int o = WR_THREADS / 2; o >= 1; o >>= 1) {
    PointIO<F>::store_xyzz(sh + threadIdx.x * XW, acc);
    __syncthreads();
    if ((int)threadIdx.x < o) acc = Xyzz<F>::add(acc, PointIO<F>::load_xyzz(sh + (threadIdx.x + o) * XW));
    __syncthreads();
  }
  if (threadIdx.x == 0) PointIO<F>::store_xyzz(win + (size_t)w * XW, acc);
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

__global__ void k_div_ceil(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t K) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (in[i] + K - 1u) / K;
}

template <class F>
typename HostOf<F>::Pt msm_run(const MsmInput& in, Workspace& ws, hipStream_t st) {
  using HP = typename HostOf<F>::Pt;
  constexpr int XW = PointIO<F>::XYZZ_WORDS;
  constexpr int CW = XW / 4;  // words per coordinate
  ZK_REQUIRE(in.nscalars < (1ull << 31) && in.npoints < (1ull << 31), "MSM too large");
  const uint32_t n = (uint32_t)in.nscalars;
  if (n == 0) return HP::inf();
  int c, nw;
  msm_choose_window(n, in.max_bits, &c, &nw);
  const uint32_t nb = 1u << (c - 1);
  const uint32_t nbt = (uint32_t)nw * nb;

  uint32_t* digits = ws.get(S_DIGITS, (size_t)nw * n * 4);
  uint32_t* counts = ws.get(S_COUNTS, (size_t)nbt * 4);
  uint32_t* offsets = ws.get(S_OFFSETS, (size_t)nbt * 4);
  uint32_t* cursor = ws.get(S_CURSOR, (size_t)nbt * 4);
  uint32_t* meta = ws.get(S_META, 64 * 4);  // [0] entries, [1] max bucket, [2] tasks, [3] max tasks/bucket
  uint32_t* cntb[2] = {ws.get(S_CNT_A, (size_t)nbt * 4), ws.get(S_CNT_B, (size_t)nbt * 4)};
  uint32_t* offb[2] = {ws.get(S_OFF_A, (size_t)nbt * 4), ws.get(S_OFF_B, (size_t)nbt * 4)};
  fill_u32(counts, 0u, nbt, st);

  DigitParams dp{in.scalars, n, in.points, (uint32_t)in.npoints, in.scalars_mont ? 1 : 0,
                 in.point_index_bitrev, c, nw, nb, digits, counts};
  {
    ProfScope ps(PointIO<F>::AFF_WORDS == 16 ? "msm_digits_g1" : "msm_digits_g2", st, (double)n);
    hipLaunchKernelGGL(k_msm_digits<F>, dim3(cdiv(n, 256)), dim3(256), 0, st, dp);
    ZK_HIP(hipGetLastError());
  }
  scan_exclusive(counts, offsets, nbt, 0, meta + 0, meta + 1, ws, S_SCRATCH, st);
  ZK_HIP(hipMemcpyAsync(cursor, offsets, (size_t)nbt * 4, hipMemcpyDeviceToDevice, st));
  uint32_t hm[2];
  ZK_HIP(hipMemcpyAsync(hm, meta, 8, hipMemcpyDeviceToHost, st));
  ZK_HIP(hipStreamSynchronize(st));
  const uint32_t total = hm[0];
  if (total == 0) return HP::inf();
  uint32_t* sorted = ws.get(S_SORTED, (size_t)total * 4);
  {
    ProfScope ps("msm_scatter", st, (double)total);
    hipLaunchKernelGGL(k_msm_scatter, dim3(cdiv(n, 256)), dim3(256), 0, st, digits, n, nw, nb, cursor, sorted,
                       in.point_index_bitrev);
    ZK_HIP(hipGetLastError());
  }

  // Accumulation levels.  Level 0 sums points; later levels sum the partial
  // sums of buckets that were split into several tasks.
  uint32_t K = std::max(4u, std::min(total / 65536u, 64u));
  const uint32_t* cur_cnt = counts;
  const uint32_t* cur_off = offsets;
  const uint32_t* in_part = nullptr;
  uint32_t level_entries = total;  // entries summed at the current level
  for (int level = 0;; level++) {
    uint32_t* task_off = offb[level & 1];
    uint32_t* next_cnt = cntb[level & 1];
    scan_exclusive(cur_cnt, task_off, nbt, K, meta + 2, meta + 3, ws, S_SCRATCH, st);
    ZK_HIP(hipMemcpyAsync(hm, meta + 2, 8, hipMemcpyDeviceToHost, st));
    ZK_HIP(hipStreamSynchronize(st));
    const uint32_t ntasks = hm[0], maxt = hm[1];
    uint2* tasks = ws.get<uint2>(S_TASKS, (size_t)ntasks * 8);
    uint32_t* out_part = ws.get(level & 1 ? S_PART1 : S_PART0, (size_t)ntasks * XW * 4);
    hipLaunchKernelGGL(k_msm_tasks, dim3(cdiv(nbt, 256)), dim3(256), 0, st, cur_cnt, cur_off, task_off, nbt, K,
                       tasks);
    ZK_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_div_ceil, dim3(cdiv(nbt, 256)), dim3(256), 0, st, cur_cnt, next_cnt, nbt, K);
    ZK_HIP(hipGetLastError());
    {
      const bool g1 = PointIO<F>::AFF_WORDS == 16;
      // work: one addition per entry summed (level 0: points; later: partials)
      ProfScope ps(level == 0 ? (g1 ? "msm_acc_points_g1" : "msm_acc_points_g2")
                              : (g1 ? "msm_acc_partials_g1" : "msm_acc_partials_g2"),
                   st, level == 0 ? (double)total : (double)level_entries);
      if (level == 0)
        hipLaunchKernelGGL(k_msm_acc_points<F>, dim3(cdiv(ntasks, 64)), dim3(64), 0, st, tasks, meta + 2, sorted,
                           in.points, out_part);
      else
        hipLaunchKernelGGL(k_msm_acc_partials<F>, dim3(cdiv(ntasks, 64)), dim3(64), 0, st, tasks, meta + 2,
                           in_part, out_part);
      ZK_HIP(hipGetLastError());
    }
    level_entries = ntasks;
    cur_cnt = next_cnt;
    cur_off = task_off;
    in_part = out_part;
    if (maxt <= 1) break;
    K = 8;
  }

  // Bucket reduction: segments of L buckets, about 32k segments in all.
  uint32_t L = 1;
  while ((size_t)nbt / L > 32768 && L < nb) L <<= 1;
  const uint32_t G = nb / L;
  uint32_t* seg = ws.get(S_SEG, (size_t)nw * G * XW * 4);
  {
    ProfScope ps(PointIO<F>::AFF_WORDS == 16 ? "msm_segments_g1" : "msm_segments_g2", st, (double)nbt);
    hipLaunchKernelGGL(k_msm_segments<F>, dim3(cdiv((size_t)nw * G, 64)), dim3(64), 0, st, cur_cnt, cur_off,
                       in_part, nw, nb, L, seg);
    ZK_HIP(hipGetLastError());
  }
  uint32_t* win = ws.get(S_WIN, (size_t)nw * XW * 4);
  {
    ProfScope ps(PointIO<F>::AFF_WORDS == 16 ? "msm_window_reduce_g1" : "msm_window_reduce_g2", st,
                 (double)nw * G);
    hipLaunchKernelGGL(k_msm_window_reduce<F>, dim3(nw), dim3(WR_THREADS), 0, st, seg, G, win);
    ZK_HIP(hipGetLastError());
  }
  std::vector<uint32_t> hw((size_t)nw * XW);
  ZK_HIP(hipMemcpyAsync(hw.data(), win, hw.size() * 4, hipMemcpyDeviceToHost, st));
  ZK_HIP(hipStreamSynchronize(st));

  // Horner over windows on the host
  HP acc = HP::inf();
  for (int w = nw - 1; w >= 0; w--) {
    if (w != nw - 1)
      for (int d = 0; d < c; d++) acc = HP::dbl(acc);
    const uint32_t* p = hw.data() + (size_t)w * XW;
    auto X = HostOf<F>::coord(p), Y = HostOf<F>::coord(p + CW), ZZ = HostOf<F>::coord(p + 2 * CW),
         ZZZ = HostOf<F>::coord(p + 3 * CW);
    acc = HP::add(acc, host::xyzz_to_jac(X, Y, ZZ, ZZZ));
  }
  return acc;
}

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
