// Pippenger's bucket method for sum_j s_j P_j over G1 and G2 (Groth16's
// A, B, L and H queries), plus fixed-base batch multiplication for key
// generation.
//
// Device pipeline for a batch of MSMs, each with its own window width c and
// nw signed windows (all steps cover every MSM of the batch):
//   1. digits:  each scalar is folded to |s| <= (r-1)/2 with a sign (s > (r-1)/2
//               becomes -(r - s)) and recoded into signed digits in
//               (-2^(c-1), 2^(c-1)]; digit d != 0 of window w names bucket
//               |d| - 1 of that window and carries the sign.
//   2. sort:    per (window, chunk of scalars) an LDS histogram of buckets;
//               an exclusive scan over (bucket, chunk) gives every chunk its
//               slots inside each bucket, and a scatter with LDS cursors
//               places (point index | sign) there (a counting sort with no
//               global atomics, so skewed digits cost nothing extra).
//   3. accumulate: every bucket is cut into tasks by its size (thread tasks
//               of K entries, wavefront tasks for heavy buckets), so work
//               stays balanced whatever the bucket sizes (small-integer
//               scalars pile into few buckets); a task sums its points with
//               mixed XYZZ additions, and a pass per bucket adds its task sums.
//   4. reduce:  bit planes: S[w c + j] = sum of the buckets whose digit value
//               has bit j set, so sum_j 2^j S[w c + j] = sum_b (b + 1) B_b.
//   5. host:    sum_q 2^q S[q] by Horner's rule (a serial chain of about 254
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
#include "tune.hpp"

namespace zkvc {

constexpr uint32_t EMPTY = 0xffffffffu;
constexpr uint32_t WG_TASK_ENTRIES = 256;  // entries per large-bucket (wavefront) task
constexpr uint32_t WG_TASK_ENTRIES_QUAD = 64;  // the same when the wavefront works in quads (latency-bound batches)
constexpr uint32_t SIGN = 0x80000000u;
enum MsmSlot {
  S_DIGITS = 100, S_COUNTS, S_OFFSETS, S_HEAVY, S_SORTED, S_TASKS, S_CNT_A, S_CNT_B, S_OFF_A, S_OFF_B,
  S_PART0, S_PART1, S_SCRATCH, S_SCRATCH2, S_SEG, S_WIN, S_META, S_FB_XYZZ, S_FB_PREFIX, S_BP_PART, S_JOBS, S_RED
};

__device__ __forceinline__ uint32_t bitrev_n(uint32_t a, int bits) {
  return bits == 0 ? 0u : (__builtin_bitreverse32(a) >> (32 - bits));
}

// ---------------------------------------------------------------- batch description
// Several MSMs over the same group run as one device pipeline: every kernel
// below covers all of them, so a batch of small MSMs still fills the device.
// Each job has its own window width and its own ranges in the shared arrays.
struct JobDev {
  const uint32_t* points;   // affine points, device layout
  const uint32_t* scalars;  // Fr elements, 8 words each
  uint32_t n, npoints;
  int mont, bitrev_bits, c, nw;
  int pre;                  // precomputed windows: window w's digits index the points of copy w
  uint32_t nb;              // buckets per window: 2^(c-1)
  uint32_t nwb;             // bucket sets: nw, or 1 with precomputed windows
  uint32_t chunk, nch;      // digits per histogram chunk and number of chunks: per window, or (with
                            // precomputed windows) over the job's whole digit stream of nw * n digits
  uint32_t digit_base;      // first digit word (nw * n words, window-major)
  uint32_t bucket_base;     // first bucket (nwb * nb buckets, window-major)
  uint32_t hist_base;       // first histogram word (nwb * nch * nb words)
  uint32_t plane_base;      // first bit plane (nwb * c planes)
  uint32_t bpb;             // blocks per bit plane (a power of two)
  uint32_t blk_bp;          // first block of the bit-plane grid (nwb * c * bpb blocks)
  // the grid reduction of large bucket sets (see k_msm_gridsums): log2 of the
  // grid's row length L (0: plain bit planes), its first sum, first block
  uint32_t grid_lg, grid_base, blk_gs;
  // bit-plane entries (the reduction table, see batch_plan): points per set
  // read from set_stride apart, log2(nb), and where set w's plane j goes:
  // plane_base + w * pstride + poff + j
  uint32_t set_stride, lg, pstride, poff;
  uint32_t blk_digits;      // first block of the digit grid
  uint32_t blk_hs;          // first block of the histogram / scatter grid (nw * nch blocks, or nch)
  // signed-digit recoding: K = sum_{w < nw} (2^(c-1) - 1) 2^(c w) (9 words:
  // c nw reaches 268 bits); digits_pw: one digit thread per (window, scalar)
  // instead of per scalar
  uint32_t kadd[9];
  uint32_t digits_pw;
};
// A batch of up to INLINE_JOBS jobs (a single proof's lanes, a single MSM)
// carries its job records in the kernel arguments; a larger batch (every
// proof of a proving batch at once) keeps them in a device table uploaded
// with the batch.  No upload means no copy on the lane's critical path.
constexpr int INLINE_JOBS = 8;
struct BatchDev {
  int njobs;
  int prio;  // 1: the batch is on the critical path (its waves win instruction issue)
  const JobDev* jobs;
  JobDev inl[INLINE_JOBS];
  __device__ __forceinline__ const JobDev& job(int k) const { return njobs <= INLINE_JOBS ? inl[k] : jobs[k]; }
};

// A critical-path batch raises its waves' issue priority over waves of
// concurrent kernels on the same SIMD (the other lanes' MSMs).
__device__ __forceinline__ void wave_priority(int prio) {
  if (prio) __builtin_amdgcn_s_setprio(2);
}

// The job owning index v of a per-job range whose first index is the field F
// (ascending over the jobs): a binary search of the table.
template <uint32_t JobDev::*F>
__device__ __forceinline__ int job_of(const BatchDev& B, uint32_t v) {
  int lo = 0, hi = B.njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (B.job(mid).*F <= v)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

constexpr int MAX_C = 15;         // the LDS histogram holds 2^(c-1) u32 counters (<= 64 KiB)
constexpr int HS_THREADS = 512;   // histogram / scatter blocks
constexpr int WG_THREADS = 64;    // one wavefront per large-bucket task (at most 4 entries per lane)
constexpr int BP_THREADS = 256;   // bit-plane reduction block
constexpr uint64_t FEW_BUCKETS = 4096;  // a wavefront per bucket leaves most of the device free
// Above this many bucket entries, thread tasks of a few entries each already
// fill the device, and their additions cost about half the VALU work of the
// cooperative forms (no idle product slots, no trees inside a task).
constexpr uint64_t FEW_ENTRIES = 1ull << 19;
constexpr uint64_t FIN_QUAD_BUCKETS = 16384;     // see batch_plan (finalize in quads)
constexpr uint64_t FIN_QUAD_LANES = 1ull << 16;  // about one wavefront per SIMD (2^17 measured 2% slower)

// ---------------------------------------------------------------- 1. digits
// Fold s > (r-1)/2 to r - s with the sign flipped, then recode into signed
// digits d_w in (-2^(c-1), 2^(c-1)] with s = sum_w d_w 2^(c w).  With the
// constant K = sum_w (2^(c-1) - 1) 2^(c w), window w of S = s + K holds
// d_w + 2^(c-1) - 1 (a window's carry into the next is exactly the carry of
// the binary addition), so every window's digit is read off S on its own.
// Output: one word per window (bucket |d| - 1 | sign, or EMPTY for a zero
// digit or a point at infinity).  Jobs with few scalars and many windows
// take a thread per (window, scalar), the others a thread per scalar.
template <class F>
__global__ void __launch_bounds__(256) k_msm_digits(BatchDev B, uint32_t* digits) {
  wave_priority(B.prio);
  const int k = job_of<&JobDev::blk_digits>(B, blockIdx.x);
  const JobDev& J = B.job(k);
  const uint32_t t = (blockIdx.x - J.blk_digits) * 256 + threadIdx.x;
  uint32_t j, w0, w1;
  if (J.digits_pw) {
    if (t >= J.n * (uint32_t)J.nw) return;
    w0 = t / J.n;
    j = t - w0 * J.n;
    w1 = w0 + 1;
  } else {
    if (t >= J.n) return;
    j = t;
    w0 = 0;
    w1 = (uint32_t)J.nw;
  }
  const uint32_t idx = J.bitrev_bits ? bitrev_n(j, J.bitrev_bits) : j;
  bool skip = idx >= J.npoints;
  if (!skip) skip = PointIO<F>::affine_is_zero(J.points + (size_t)idx * PointIO<F>::AFF_WORDS);
  uint32_t s[9];
  {
    const uint4 a = reinterpret_cast<const uint4*>(J.scalars + 8ull * j)[0];
    const uint4 b = reinterpret_cast<const uint4*>(J.scalars + 8ull * j)[1];
    s[0] = a.x; s[1] = a.y; s[2] = a.z; s[3] = a.w; s[4] = b.x; s[5] = b.y; s[6] = b.z; s[7] = b.w;
    s[8] = 0u;
  }
  if (J.mont) {
    Fr x = Fr::unpack(s);
    x = Fr::from_mont(x);
    x.pack(s);
  }
  bool gt = false, decided = false;
#pragma unroll
  for (int q = 7; q >= 0; q--) {
    if (!decided && s[q] != FrParams::HALF32[q]) {
      gt = s[q] > FrParams::HALF32[q];
      decided = true;
    }
  }
  const uint32_t neg = gt ? 1u : 0u;
  if (gt) {
    uint64_t borrow = 0;
#pragma unroll
    for (int q = 0; q < 8; q++) {
      const uint64_t d = (uint64_t)FrParams::P32[q] - s[q] - borrow;
      s[q] = (uint32_t)d;
      borrow = (d >> 32) & 1u;
    }
  }
  // S = s + K (below 2^(c nw): s < 2^(c nw - 1) and K < 2^(c nw - 1))
  {
    uint64_t carry = 0;
#pragma unroll
    for (int q = 0; q < 9; q++) {
      const uint64_t a = (uint64_t)s[q] + J.kadd[q] + carry;
      s[q] = (uint32_t)a;
      carry = a >> 32;
    }
  }
  const int c = J.c;
  const int32_t bias = (int32_t)(1u << (c - 1)) - 1;
  const uint32_t cmask = (1u << c) - 1u;
  uint32_t* out = digits + J.digit_base + j;
  for (uint32_t w = w0; w < w1; w++) {
    const int pos = c * (int)w;
    const int q = pos >> 5, sh = pos & 31;
    uint32_t raw = 0;
    if (q < 9) {
      const uint32_t lo = s[q];
      const uint32_t hi = q + 1 < 9 ? s[q + 1] : 0u;
      raw = (uint32_t)((((uint64_t)hi << 32) | lo) >> sh) & cmask;
    }
    const int32_t d = (int32_t)raw - bias;
    const uint32_t sgn = d < 0 ? 1u : 0u;
    const uint32_t mag = (uint32_t)(d < 0 ? -d : d);
    out[(size_t)w * J.n] = (!skip && mag != 0u) ? ((mag - 1u) | ((neg ^ sgn) << 31)) : EMPTY;
  }
}

// ---------------------------------------------------------------- 2. counting sort
// Block (window w, chunk ch) counts its digits per bucket in LDS and writes
// the counts as one contiguous row, hist[(w nch + ch) nb + b].  With
// precomputed windows all windows share one bucket set and a block takes
// chunk ch of the job's whole digit stream (window-major, nw n digits):
// hist[ch nb + b].  A thread per bucket then walks its column of rows
// (k_msm_colscan), turning the counts into the bucket's running offsets per
// chunk and its total; a scan of the totals gives each bucket its first slot.
// Every access is coalesced and no global atomics are used, however skewed
// the digits are.
struct HsRange {
  const uint32_t* d;  // the block's digits: d[lo .. hi)
  uint32_t lo, hi;
  size_t row;         // its histogram row (bucket b at row + b)
  uint32_t w;         // its window's bucket set (0 with precomputed windows)
};
__device__ __forceinline__ HsRange hs_range(const JobDev& J, const uint32_t* digits, uint32_t local) {
  HsRange r;
  if (J.pre) {
    const uint32_t total = (uint32_t)J.nw * J.n;
    r.d = digits + J.digit_base;
    r.lo = local * J.chunk;
    r.hi = min(total, r.lo + J.chunk);
    r.row = (size_t)J.hist_base + (size_t)local * J.nb;
    r.w = 0;
  } else {
    const uint32_t w = local / J.nch, ch = local % J.nch;
    r.d = digits + J.digit_base + (size_t)w * J.n;
    r.lo = ch * J.chunk;
    r.hi = min(J.n, r.lo + J.chunk);
    r.row = (size_t)J.hist_base + ((size_t)w * J.nch + ch) * J.nb;
    r.w = w;
  }
  return r;
}
__global__ void __launch_bounds__(HS_THREADS) k_msm_hist(BatchDev B, const uint32_t* digits, uint32_t* hist) {
  wave_priority(B.prio);
  extern __shared__ uint32_t cnt[];
  const int k = job_of<&JobDev::blk_hs>(B, blockIdx.x);
  const JobDev& J = B.job(k);
  const HsRange R = hs_range(J, digits, blockIdx.x - J.blk_hs);
  for (uint32_t b = threadIdx.x; b < J.nb; b += HS_THREADS) cnt[b] = 0u;
  __syncthreads();
  for (uint32_t i = R.lo + threadIdx.x; i < R.hi; i += HS_THREADS) {
    const uint32_t v = R.d[i];
    if (v != EMPTY) atomicAdd(&cnt[v & ~SIGN], 1u);
  }
  __syncthreads();
  uint32_t* h = hist + R.row;
  for (uint32_t b = threadIdx.x; b < J.nb; b += HS_THREADS) h[b] = cnt[b];
}

// A group of G lanes (G = 4 or 8, a power of two dividing the wavefront)
// per bucket f (window w, digit value b): lane q of the group takes the q-th
// share of the bucket's column of histogram rows.  A first pass sums each
// share, a scan across the group gives each share its start, and a second
// pass turns the counts into running offsets inside the bucket, in place;
// cnt[f] receives the bucket's size and nt[f] its number of tasks (see
// k_msm_make_tasks).  Also clears the task-list counters.
__global__ void __launch_bounds__(256) k_msm_colscan(BatchDev B, uint32_t* hist, uint32_t nbt, uint32_t K,
                                                     uint32_t large, uint32_t wg_entries, uint32_t* cnt, uint32_t* nt,
                                                     uint32_t* counters, uint32_t lg_group) {
  wave_priority(B.prio);
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t G = 1u << lg_group;
  const uint32_t f = t >> lg_group, q = t & (G - 1u);
  if (t == 0) {
    counters[0] = 0u;
    counters[1] = 0u;
    counters[2] = 0u;
  }
  // a group's lanes share f: the whole group is in or out
  if (f >= nbt) return;
  const int k = job_of<&JobDev::bucket_base>(B, f);
  const JobDev& J = B.job(k);
  const uint32_t lf = f - J.bucket_base;
  const uint32_t w = lf / J.nb, b = lf - w * J.nb;
  const uint32_t nch = J.nch, nb = J.nb;
  const uint32_t per = (nch + G - 1) >> lg_group;
  const uint32_t c0 = min(nch, q * per), c1 = min(nch, c0 + per);
  uint32_t* col = hist + J.hist_base + (size_t)w * nch * nb + b;
  uint32_t part = 0;
#pragma unroll 8
  for (uint32_t ch = c0; ch < c1; ch++) part += col[(size_t)ch * nb];
  // inclusive scan of the share sums inside the group (lanes of a group are
  // consecutive and aligned inside the wavefront)
  uint32_t inc = part;
  for (uint32_t o = 1; o < G; o <<= 1) {
    const uint32_t v = __shfl_up(inc, o, 64);
    if (q >= o) inc += v;
  }
  const uint32_t total = __shfl(inc, (threadIdx.x & 63u) | (G - 1u), 64);
  uint32_t run = inc - part;
#pragma unroll 8
  for (uint32_t ch = c0; ch < c1; ch++) {
    const uint32_t v = col[(size_t)ch * nb];
    col[(size_t)ch * nb] = run;
    run += v;
  }
  if (q == 0) {
    cnt[f] = total;
    const uint32_t sz = total >= large ? wg_entries : K;
    nt[f] = (total + sz - 1) / sz;
  }
}

// Same blocks as k_msm_hist: LDS cursors start at the bucket's first slot
// plus the chunk's running offset inside the bucket, and every digit takes the
// next slot of its bucket (order inside a bucket does not matter to the sum).  Entries are (point index | sign); with
// precomputed windows stream position p holds window p / n of scalar p % n,
// whose point is copy p / n of the scalar's base.
__global__ void __launch_bounds__(HS_THREADS) k_msm_scatter(BatchDev B, const uint32_t* digits, const uint32_t* hist,
                                                            const uint32_t* off, uint32_t* sorted) {
  wave_priority(B.prio);
  extern __shared__ uint32_t cur[];
  const int k = job_of<&JobDev::blk_hs>(B, blockIdx.x);
  const JobDev& J = B.job(k);
  const HsRange R = hs_range(J, digits, blockIdx.x - J.blk_hs);
  const uint32_t* h = hist + R.row;
  const uint32_t* o = off + J.bucket_base + (size_t)R.w * J.nb;
  for (uint32_t b = threadIdx.x; b < J.nb; b += HS_THREADS) cur[b] = o[b] + h[b];
  __syncthreads();
  for (uint32_t p = R.lo + threadIdx.x; p < R.hi; p += HS_THREADS) {
    const uint32_t v = R.d[p];
    if (v == EMPTY) continue;
    const uint32_t pos = atomicAdd(&cur[v & ~SIGN], 1u);
    uint32_t i = p, pbase = 0u;
    if (J.pre) {
      const uint32_t w = p / J.n;
      i = p - w * J.n;
      pbase = w * J.npoints;
    }
    const uint32_t idx = J.bitrev_bits ? bitrev_n(i, J.bitrev_bits) : i;
    sorted[pos] = (pbase + idx) | (v & SIGN);
  }
}

// ---------------------------------------------------------------- 3. tasks and accumulation
// Buckets are split into tasks by their actual size: a bucket with fewer than
// `large` entries becomes thread tasks of at most K entries (one thread sums a
// task serially); a larger one becomes wavefront tasks of WG_TASK_ENTRIES
// entries reduced by an LDS tree.  nt[f] (from k_msm_colscan) is the number
// of partial sums of bucket f; a bucket's partial sums are contiguous.

// Task records (first entry, length, output partial slot, job).  Slots in
// the two task lists are claimed with one atomic per wavefront and list.
// Buckets that end up with more than `fin_max` partial sums (several times
// the batch's average, at least FIN_THREAD_MIN) are listed for a wavefront
// each in the finalize step; the others are summed by one thread each.
constexpr uint32_t FIN_THREAD_MIN = 8;

__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t v, uint32_t lane) {
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t a = __shfl_up(v, o, 64);
    if ((int)lane >= o) v += a;
  }
  return v;
}

__global__ void __launch_bounds__(256) k_msm_make_tasks(BatchDev B, const uint32_t* cnt, const uint32_t* off,
                                                        const uint32_t* part_off, uint32_t nbt, uint32_t K,
                                                        uint32_t large, uint32_t wg_entries, uint32_t fin_max,
                                                        uint32_t* counters, uint4* th_tasks, uint4* wg_tasks,
                                                        uint32_t* heavy) {
  wave_priority(B.prio);
  const uint32_t f = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t c = f < nbt ? cnt[f] : 0u;
  const bool big = c >= large;
  const uint32_t sz = big ? wg_entries : K;
  const uint32_t nt = (c + sz - 1) / sz;
  const uint32_t hv = nt > fin_max ? 1u : 0u;
  // inclusive wavefront scans of the three claims
  const uint32_t sth = wave_inclusive_sum(big ? 0u : nt, lane);
  const uint32_t swg = wave_inclusive_sum(big ? nt : 0u, lane);
  const uint32_t shv = wave_inclusive_sum(hv, lane);
  uint32_t bth = 0, bwg = 0, bhv = 0;
  if (lane == 63u) {
    if (sth) bth = atomicAdd(&counters[0], sth);
    if (swg) bwg = atomicAdd(&counters[1], swg);
    if (shv) bhv = atomicAdd(&counters[2], shv);
  }
  bth = __shfl(bth, 63, 64);
  bwg = __shfl(bwg, 63, 64);
  bhv = __shfl(bhv, 63, 64);
  if (c == 0) return;
  if (hv) heavy[bhv + shv - 1u] = f;
  const uint32_t base = big ? bwg + swg - nt : bth + sth - nt;
  uint4* dst = big ? wg_tasks : th_tasks;
  const uint32_t o = off[f], p = part_off[f];
  const uint32_t job = (uint32_t)job_of<&JobDev::bucket_base>(B, f);
  for (uint32_t q = 0; q < nt; q++) {
    const uint32_t len = c - q * sz < sz ? c - q * sz : sz;
    dst[base + q] = make_uint4(o + q * sz, len, p + q, job);
  }
}

// The sum over nteams quads of their values (each quad's four lanes hold the
// same point): an LDS tree of cooperative additions.  Every thread of the
// block must call; the result is valid in quad 0.
template <class F>
__device__ __forceinline__ Xyzz<F> quad_tree_sum(Xyzz<F> acc, uint32_t* sh, uint32_t nteams) {
  constexpr int XW = PointIO<F>::XYZZ_WORDS;
  const uint32_t team = threadIdx.x >> 2, tq = threadIdx.x & 3u;
  for (uint32_t o = nteams / 2; o >= 1; o >>= 1) {
    if (team >= o && team < 2 * o && tq == 0) PointIO<F>::store_xyzz(sh + (team - o) * XW, acc);
    __syncthreads();
    if (team < o) acc = QuadOps<F>::add(acc, PointIO<F>::load_xyzz(sh + team * XW), tq);
    __syncthreads();
  }
  return acc;
}

// Bucket accumulation, one launch for both task lists: blocks below
// th_blocks run thread tasks (each thread sums its entries serially), the
// others run wavefront tasks (each lane sums a strided share of the task's
// entries, then an LDS tree).  Task counts are read on the device; every
// loop is bounded by them.
// Waves per SIMD the accumulation and finalize kernels are built for.  The G2
// kernels would otherwise take ~370 registers, one wave per SIMD: a wave then
// holds a whole SIMD, next to the critical path's kernels, for its lifetime.
// Two waves (256 registers, a few hundred bytes of spill) measured faster
// for the proofs and for the G2 MSMs themselves; three spill too much.
template <class F>
struct AccWaves {
  static constexpr int value = sizeof(F) <= 64 ? 1 : 2;
};
template <class F>
__global__ void __launch_bounds__(64, AccWaves<F>::value) k_msm_acc(BatchDev B, const uint4* th_tasks, const uint4* wg_tasks,
                                                const uint32_t* counters, uint32_t th_blocks, const uint32_t* sorted,
                                                uint32_t* partials, int quad, const uint32_t* total,
                                                uint32_t* work_out) {
  wave_priority(B.prio);
  constexpr int XW = PointIO<F>::XYZZ_WORDS;
  constexpr int AW = PointIO<F>::AFF_WORDS;
  __shared__ uint32_t sh[WG_THREADS / 2 * XW];
  if (work_out && blockIdx.x == 0 && threadIdx.x == 0) {  // the work count for a profile (host memory)
    *work_out = *total;
    __threadfence_system();
  }
  if (blockIdx.x < th_blocks) {
    const uint32_t ntasks = counters[0];
    for (uint32_t t = blockIdx.x * 64 + threadIdx.x; t < ntasks; t += th_blocks * 64) {
      const uint4 task = th_tasks[t];
      const uint32_t* points = B.job(task.w).points;
      Xyzz<F> acc = Xyzz<F>::inf();
      // the next entry's point is loaded while the current one is added
      const uint32_t end = task.x + task.y;
      uint32_t ref = sorted[task.x];
      Affine<F> pt = PointIO<F>::load_affine(points + (size_t)(ref & ~SIGN) * AW);
      for (uint32_t e = task.x; e < end; e++) {
        Affine<F> cur = pt;
        const uint32_t cref = ref;
        if (e + 1 < end) {
          ref = sorted[e + 1];
          pt = PointIO<F>::load_affine(points + (size_t)(ref & ~SIGN) * AW);
        }
        if (cref & SIGN) cur.y = F::neg_canon_lz(cur.y);  // stored coordinates are canonical
        acc = Xyzz<F>::madd(acc, cur);
      }
      PointIO<F>::store_xyzz(partials + (size_t)task.z * XW, acc);
    }
    return;
  }
  const uint32_t ntasks = counters[1];  // uniform: every lane of the block runs the same loop count
  const uint32_t wg_blocks = gridDim.x - th_blocks;
  const uint32_t team = threadIdx.x >> 2, tq = threadIdx.x & 3u;
  for (uint32_t t = blockIdx.x - th_blocks; t < ntasks; t += wg_blocks) {
    const uint4 task = wg_tasks[t];
    const uint32_t* points = B.job(task.w).points;
    Xyzz<F> acc = Xyzz<F>::inf();
    if (quad) {
      // 16 quads, each summing a strided share with cooperative additions
      for (uint32_t e = team; e < task.y; e += WG_THREADS / 4) {
        const uint32_t ref = sorted[task.x + e];
        Affine<F> pt = PointIO<F>::load_affine(points + (size_t)(ref & ~SIGN) * AW);
        if (ref & SIGN) pt.y = F::neg_canon_lz(pt.y);
        acc = QuadOps<F>::madd(acc, pt, tq);
      }
      acc = quad_tree_sum<F>(acc, sh, WG_THREADS / 4);
    } else {
      for (uint32_t e = threadIdx.x; e < task.y; e += WG_THREADS) {
        const uint32_t ref = sorted[task.x + e];
        Affine<F> pt = PointIO<F>::load_affine(points + (size_t)(ref & ~SIGN) * AW);
        if (ref & SIGN) pt.y = F::neg_canon_lz(pt.y);
        acc = Xyzz<F>::madd(acc, pt);
      }
      for (int o = WG_THREADS / 2; o >= 1; o >>= 1) {
        if ((int)threadIdx.x >= o && (int)threadIdx.x < 2 * o) PointIO<F>::store_xyzz(sh + (threadIdx.x - o) * XW, acc);
        __syncthreads();
        if ((int)threadIdx.x < o) acc = Xyzz<F>::add(acc, PointIO<F>::load_xyzz(sh + threadIdx.x * XW));
        __syncthreads();
      }
    }
    if (threadIdx.x == 0) PointIO<F>::store_xyzz(partials + (size_t)task.z * XW, acc);
  }
}

// Bucket sums from the partial sums, one launch: blocks below light_blocks
// give each bucket with at most fin_max partials a group of `group` lanes
// (a power of two <= 64; each lane, or each quad with quad set, sums a
// strided share, then a tree over the group); the others give each listed
// heavy bucket a wavefront (strided sums, then a tree), so one crowded bucket
// (e.g. the top window's few digit values under uniform scalars) does not
// serialize the step.  quad: latency-bound batches add in cooperative quads.
template <class F>
__global__ void __launch_bounds__(64, AccWaves<F>::value) k_msm_finalize(const uint32_t* nt, const uint32_t* part_off,
                                                     const uint32_t* partials, uint32_t nbt, const uint32_t* counters,
                                                     const uint32_t* heavy, uint32_t light_blocks, uint32_t fin_max,
                                                     uint32_t group, int quad, uint32_t* buckets, int prio) {
  wave_priority(prio);
  constexpr int XW = PointIO<F>::XYZZ_WORDS;
  __shared__ uint32_t sh[WG_THREADS * XW];
  const uint32_t tq = threadIdx.x & 3u;
  if (blockIdx.x < light_blocks) {
    const uint32_t f = blockIdx.x * (WG_THREADS / group) + threadIdx.x / group;
    const uint32_t lane = threadIdx.x & (group - 1u);
    uint32_t c = 0, o = 0;
    if (f < nbt) {
      c = nt[f];
      o = part_off[f];
    }
    const bool mine = f < nbt && c <= fin_max;
    Xyzz<F> acc = Xyzz<F>::inf();
    if (quad) {  // group >= 4: group / 4 quads per bucket
      const uint32_t qi = lane >> 2, nq = group >> 2;
      if (mine)
        for (uint32_t e = qi; e < c; e += nq)
          acc = QuadOps<F>::add(acc, PointIO<F>::load_xyzz(partials + (size_t)(o + e) * XW), tq);
      for (uint32_t q = nq / 2; q >= 1; q >>= 1) {  // every thread of the block takes part
        if (qi >= q && qi < 2 * q && tq == 0) PointIO<F>::store_xyzz(sh + (threadIdx.x / 4 - q) * XW, acc);
        __syncthreads();
        if (qi < q) acc = QuadOps<F>::add(acc, PointIO<F>::load_xyzz(sh + (threadIdx.x / 4) * XW), tq);
        __syncthreads();
      }
    } else {
      if (mine)
        for (uint32_t e = lane; e < c; e += group)
          acc = Xyzz<F>::add(acc, PointIO<F>::load_xyzz(partials + (size_t)(o + e) * XW));
      for (uint32_t q = group / 2; q >= 1; q >>= 1) {  // every thread of the block takes part
        if (lane >= q && lane < 2 * q) PointIO<F>::store_xyzz(sh + (threadIdx.x - q) * XW, acc);
        __syncthreads();
        if (lane < q) acc = Xyzz<F>::add(acc, PointIO<F>::load_xyzz(sh + threadIdx.x * XW));
        __syncthreads();
      }
    }
    if (mine && lane == 0) PointIO<F>::store_xyzz(buckets + (size_t)f * XW, acc);
    return;
  }
  const uint32_t nheavy = counters[2];
  const uint32_t hblocks = gridDim.x - light_blocks;
  for (uint32_t h = blockIdx.x - light_blocks; h < nheavy; h += hblocks) {
    const uint32_t f = heavy[h];
    const uint32_t c = nt[f], o = part_off[f];
    Xyzz<F> acc = Xyzz<F>::inf();
    if (quad) {
      for (uint32_t e = threadIdx.x >> 2; e < c; e += WG_THREADS / 4)
        acc = QuadOps<F>::add(acc, PointIO<F>::load_xyzz(partials + (size_t)(o + e) * XW), tq);
      acc = quad_tree_sum<F>(acc, sh, WG_THREADS / 4);
    } else {
      for (uint32_t e = threadIdx.x; e < c; e += WG_THREADS)
        acc = Xyzz<F>::add(acc, PointIO<F>::load_xyzz(partials + (size_t)(o + e) * XW));
      for (int q = WG_THREADS / 2; q >= 1; q >>= 1) {
        if ((int)threadIdx.x >= q && (int)threadIdx.x < 2 * q) PointIO<F>::store_xyzz(sh + (threadIdx.x - q) * XW, acc);
        __syncthreads();
        if ((int)threadIdx.x < q) acc = Xyzz<F>::add(acc, PointIO<F>::load_xyzz(sh + threadIdx.x * XW));
        __syncthreads();
      }
    }
    if (threadIdx.x == 0) PointIO<F>::store_xyzz(buckets + (size_t)f * XW, acc);
  }
}

// ---------------------------------------------------------------- 4. bucket reduction
// For window w and bit j,
//   S[w c + j] = sum of B_{v-1} over the digit values v in [1, nb] with bit j set,
// so that window w contributes sum_j 2^j S[w c + j] = sum_v v B_{v-1}; the
// host adds the planes by Horner's rule.
//
// Grid reduction (bucket sets of nb >= GRID_MIN_NB).  With v = r L + l
// (L = 2^grid_lg, R = nb / L; r in [0, R], l in [0, L)),
//   sum_v v B_{v-1} = L sum_{r=1..R} r T_r + sum_{l=1..L-1} l C_l,
// where the row sum T_r adds the buckets with v in [r L, r L + L) and the
// column sum C_l those with v = l, L + l, ..., (R-1) L + l.  k_msm_gridsums
// forms the R + L - 1 sums (about 2 nb additions in trees of depth
// log2 L + 1, instead of the c nb / 2 of the bit planes over all buckets),
// and the planes are then taken over the sums: planes 0 .. grid_lg - 1 of
// the set from the column sums (digit value l), planes grid_lg .. c - 1 from
// the row sums (digit value r), which is the same plane S[w c + j] as above.
constexpr uint32_t GRID_MIN_NB = 1024;

// One block per sum: (set w, index i); i < L - 1 is column l = i + 1 (into
// slot i of the set's L + R sums), i >= L - 1 row r = i - L + 2 (into slot
// L + r - 1).  Quads add a strided share, then a tree of quads.
template <class F>
__global__ void __launch_bounds__(BP_THREADS) k_msm_gridsums(BatchDev B, uint32_t* buckets) {
  wave_priority(B.prio);
  constexpr int XW = PointIO<F>::XYZZ_WORDS;
  __shared__ uint32_t sh[BP_THREADS / 8 * XW];
  const int k = job_of<&JobDev::blk_gs>(B, blockIdx.x);
  const JobDev& J = B.job(k);
  const uint32_t L = 1u << J.grid_lg, R = J.nb >> J.grid_lg;
  const uint32_t local = blockIdx.x - J.blk_gs;
  const uint32_t w = local / (L - 1 + R), i = local % (L - 1 + R);
  const uint32_t* bw = buckets + ((size_t)J.bucket_base + (size_t)w * J.nb) * XW;
  // entry e of the sum is bucket first + e * step (digit value first + 1 + e * step)
  uint32_t first, step, count, slot;
  if (i < L - 1) {
    first = i;  // value l = i + 1
    step = L;
    count = R;
    slot = i;
  } else {
    const uint32_t r = i - (L - 1) + 1;
    first = r * L - 1;  // value r L
    step = 1;
    count = r < R ? L : 1u;  // row R holds only v = nb
    slot = L + r - 1;
  }
  const uint32_t team = threadIdx.x >> 2, tq = threadIdx.x & 3u, nteams = blockDim.x >> 2;
  Xyzz<F> acc = Xyzz<F>::inf();
  for (uint32_t e = team; e < count; e += nteams)
    acc = QuadOps<F>::add(acc, PointIO<F>::load_xyzz(bw + (size_t)(first + e * step) * XW), tq);
  acc = quad_tree_sum<F>(acc, sh, nteams);
  if (threadIdx.x == 0)
    PointIO<F>::store_xyzz(buckets + ((size_t)J.grid_base + (size_t)w * (L + R) + slot) * XW, acc);
}

// Bit planes over the entries of the reduction table: plain jobs (their
// buckets) and, for grid jobs, two entries over the column and row sums.
// A plane is split over bpb blocks; each quad of a block sums a strided
// share of its block's slice with cooperative additions, a tree of quads
// sums the block, and k_msm_plane_sums adds the bpb block sums of each plane.
// G1 bit planes run at four wavefronts per SIMD (at most 128 VGPRs, a few
// spilled): the reduction of a large bucket set then fits the device in one
// round of blocks.  G2's working set is too large for that: two waves (as
// for its accumulation, see AccWaves).
template <class F>
struct BpWaves {
  static constexpr int value = sizeof(F) <= 64 ? 4 : 2;
};
template <class F>
__global__ void __launch_bounds__(BP_THREADS, BpWaves<F>::value) k_msm_bitplanes(BatchDev B, const uint32_t* buckets, uint32_t* part,
                                                               uint32_t* S) {
  wave_priority(B.prio);
  constexpr int XW = PointIO<F>::XYZZ_WORDS;
  __shared__ uint32_t sh[BP_THREADS / 8 * XW];
  const int k = job_of<&JobDev::blk_bp>(B, blockIdx.x);
  const JobDev& J = B.job(k);
  const uint32_t local = blockIdx.x - J.blk_bp;
  const uint32_t q = local / J.bpb, slice = local % J.bpb;
  const uint32_t c = (uint32_t)J.c, nb = J.nb;
  const uint32_t w = q / c, j = q % c;
  const uint32_t* bw = buckets + ((size_t)J.bucket_base + (size_t)w * J.set_stride) * XW;
  // digit values v in [1, nb] with bit j set: v = ((t >> j) << (j + 1)) | 2^j | (t & (2^j - 1))
  const uint32_t jmask = (1u << j) - 1u;
  const uint32_t count = j < J.lg ? nb / 2 : 1u;  // bit lg = log2(nb) is set only in v = nb
  const uint32_t per = (count + J.bpb - 1) / J.bpb;
  const uint32_t t0 = slice * per, t1 = min(count, t0 + per);
  const uint32_t team = threadIdx.x >> 2, tq = threadIdx.x & 3u, nteams = blockDim.x >> 2;
  Xyzz<F> acc = Xyzz<F>::inf();
  for (uint32_t t = t0 + team; t < t1; t += nteams) {
    const uint32_t v = ((t >> j) << (j + 1)) | (1u << j) | (t & jmask);
    if (v > nb) continue;
    acc = QuadOps<F>::add(acc, PointIO<F>::load_xyzz(bw + (size_t)(v - 1) * XW), tq);
  }
  acc = quad_tree_sum<F>(acc, sh, nteams);
  if (threadIdx.x != 0) return;
  if (J.bpb == 1) {  // the block's sum is the plane
    PointIO<F>::store_xyzz(S + ((size_t)J.plane_base + (size_t)w * J.pstride + J.poff + j) * XW, Xyzz<F>::canon(acc));
    __threadfence_system();  // S may be host memory
  } else {
    PointIO<F>::store_xyzz(part + (size_t)blockIdx.x * XW, acc);
  }
}

// One wavefront (16 quads) per plane: the sum of the plane's bpb block sums.
template <class F>
__global__ void __launch_bounds__(64) k_msm_plane_sums(BatchDev B, const uint32_t* part, uint32_t* S) {
  wave_priority(B.prio);
  constexpr int XW = PointIO<F>::XYZZ_WORDS;
  __shared__ uint32_t sh[8 * XW];
  const int k = job_of<&JobDev::plane_base>(B, blockIdx.x);
  const JobDev& J = B.job(k);
  if (J.bpb == 1) return;  // written by k_msm_bitplanes
  const uint32_t q = blockIdx.x - J.plane_base;
  const uint32_t* pp = part + ((size_t)J.blk_bp + (size_t)q * J.bpb) * XW;
  const uint32_t tq = threadIdx.x & 3u;
  Xyzz<F> acc = Xyzz<F>::inf();
  for (uint32_t t = threadIdx.x >> 2; t < J.bpb; t += 16)
    acc = QuadOps<F>::add(acc, PointIO<F>::load_xyzz(pp + (size_t)t * XW), tq);
  acc = quad_tree_sum<F>(acc, sh, 16);
  if (threadIdx.x == 0) {
    PointIO<F>::store_xyzz(S + (size_t)blockIdx.x * XW, Xyzz<F>::canon(acc));
    __threadfence_system();  // S may be host memory
  }
}

// ---------------------------------------------------------------- host driver
void msm_choose_window(size_t n, int bits, int* c_out, int* nw_out) {
  if (bits < 1) bits = 1;
  double best = 1e300;
  int bc = 2, bnw = (bits + 2) / 2;
  for (int c = 2; c <= MAX_C; c++) {
    const int nw = (bits + 1 + c - 1) / c;
    const double nb = (double)(1u << (c - 1));
    // mixed additions for the entries, a pass over every bucket, and the
    // bit-plane reduction (c nb / 2 full additions per window, ~1.4 mixed each)
    const double cost = (double)n * nw + 0.5 * nw * nb + 1.4 * nw * c * nb / 2;
    if (cost < best) {
      best = cost;
      bc = c;
      bnw = nw;
    }
  }
  *c_out = bc;
  *nw_out = bnw;
}

void msm_choose_precomputed(size_t n, int bits, int max_copies, int* c_out, int* nw_out) {
  if (bits < 1) bits = 1;
  int c0, nw0;
  msm_choose_window(n, bits, &c0, &nw0);
  double best = (double)n * nw0 + 0.5 * nw0 * (double)(1u << (c0 - 1)) + 1.4 * nw0 * c0 * (double)(1u << (c0 - 1)) / 2;
  int bc = c0, bnw = 1;
  if (nw0 == 1) {
    *c_out = c0;
    *nw_out = 1;
    return;
  }
  for (int c = 2; c <= MAX_C; c++) {
    const int nw = (bits + 1 + c - 1) / c;
    if (nw > max_copies) continue;
    const double nb = (double)(1u << (c - 1));
    // one bucket set: entries, a pass over the buckets, one bit-plane reduction
    const double cost = (double)n * nw + 0.5 * nb + 1.4 * c * nb / 2;
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

// Sizes of one batch, all known on the host before any launch, so the device
// pipeline needs no host synchronization until the window sums come back.
struct BatchPlan {
  std::vector<JobDev> jobs;   // the device table's contents
  std::vector<JobDev> red;    // the reduction table: the bit-plane entries (see k_msm_bitplanes)
  std::vector<int> map;       // table entry -> caller's job
  uint64_t ngrid = 0;         // grid sums after the nbt buckets in the bucket buffer
  uint64_t gs_blocks = 0;     // blocks of k_msm_gridsums
  uint32_t gs_threads = 64;
  uint64_t ndigits = 0, nbt = 0, nh = 0, nplanes = 0, digit_blocks = 0, hs_blocks = 0, bp_blocks = 0;
  uint32_t max_nb = 0;
  uint32_t max_nch = 0;  // the largest number of histogram chunks of one bucket set
  uint32_t K = 0;      // entries per thread task
  uint32_t large = 0;  // buckets with at least this many entries get wavefront tasks
  uint64_t max_th_tasks = 0, max_wg_tasks = 0, max_partials = 0;
  uint32_t fin_max = 0;  // partial sums above which a bucket gets a wavefront in the finalize step
  uint32_t fin_group = 1;  // lanes per bucket below that (about four partial sums per lane, or two per quad)
  bool quad = false;       // latency-bound batch: wavefront tasks add in cooperative quads
  bool fin_quad = false;   // the finalize step adds in cooperative quads
  uint32_t wg_entries = WG_TASK_ENTRIES;
};

static BatchPlan batch_plan(const MsmInput* in, int njobs, int group) {
  BatchPlan p;
  for (int q = 0; q < njobs; q++) {
    ZK_REQUIRE(in[q].nscalars < (1ull << 31) && in[q].npoints < (1ull << 31), "MSM too large");
    if (in[q].nscalars == 0) continue;
    p.jobs.emplace_back();
    JobDev& J = p.jobs.back();
    J.points = in[q].points;
    J.scalars = in[q].scalars;
    J.n = (uint32_t)in[q].nscalars;
    J.npoints = (uint32_t)in[q].npoints;
    J.mont = in[q].scalars_mont ? 1 : 0;
    J.bitrev_bits = in[q].point_index_bitrev;
    if (in[q].pre_c > 0) {
      ZK_REQUIRE(in[q].pre_c >= 2 && in[q].pre_c <= MAX_C && in[q].pre_nw >= 1 &&
                     in[q].pre_c * in[q].pre_nw >= in[q].max_bits + 1 &&
                     (uint64_t)in[q].npoints * in[q].pre_nw < (1ull << 31),
                 "invalid precomputed MSM windows");
      J.c = in[q].pre_c;
      J.nw = in[q].pre_nw;
      J.pre = 1;
    } else {
      msm_choose_window(J.n, in[q].max_bits, &J.c, &J.nw);
      // a tuned width for wide scalars of this size, if the autotuner picked one
      const int tc = in[q].max_bits > 64 && in[q].use_tuning
                         ? tuning().msm_c[group][std::min(32, ceil_log2(J.n))].load() : 0;
      if (tc >= 2 && tc <= MAX_C) {
        J.c = tc;
        J.nw = (in[q].max_bits + 1 + tc - 1) / tc;
      }
      J.pre = 0;
    }
    J.nb = 1u << (J.c - 1);
    J.nwb = J.pre ? 1u : (uint32_t)J.nw;
    {  // K = sum_w (2^(c-1) - 1) 2^(c w), c nw <= 256 bits
      uint64_t kw[5] = {0, 0, 0, 0, 0};
      for (int w = 0; w < J.nw; w++) {
        const int pos = J.c * w, q = pos >> 6, sh = pos & 63;
        const uint64_t v = (1ull << (J.c - 1)) - 1ull;
        // add v << pos into the 256-bit value (no overflow: K < 2^(c nw - 1))
        unsigned __int128 acc = (unsigned __int128)v << sh;
        for (int i = q; i < 5 && acc; i++) {
          acc += kw[i];
          kw[i] = (uint64_t)acc;
          acc >>= 64;
        }
      }
      for (int i = 0; i < 4; i++) {
        J.kadd[2 * i] = (uint32_t)kw[i];
        J.kadd[2 * i + 1] = (uint32_t)(kw[i] >> 32);
      }
      J.kadd[8] = (uint32_t)kw[4];
      ZK_REQUIRE((kw[4] >> 32) == 0, "MSM window layout beyond 288 bits");
    }
    // few scalars, many windows: spread the recoding over (window, scalar)
    J.digits_pw = J.nw >= 4 && J.n < 16384 ? 1u : 0u;
    const uint64_t wb = (uint64_t)J.nw * J.nb;
    if (J.pre) {
      // one bucket set: chunks of >= 4096 digits over the whole stream (a
      // block per chunk: enough blocks to spread the sort over the device),
      // at most 2^22 histogram words
      const uint64_t total = (uint64_t)J.nw * J.n;
      const uint64_t nch = std::max<uint64_t>(1, std::min<uint64_t>((total + 4095) / 4096, (1ull << 22) / J.nb));
      const uint64_t chunk = ((total + nch - 1) / nch + 255) / 256 * 256;
      J.chunk = (uint32_t)chunk;
      J.nch = (uint32_t)((total + chunk - 1) / chunk);
    } else {
      // chunks of >= 4096 scalars per window, at most 2^22 histogram words
      const uint64_t nch = std::max<uint64_t>(1, std::min<uint64_t>((J.n + 4095) / 4096, (1ull << 22) / wb));
      const uint64_t chunk = ((J.n + nch - 1) / nch + 255) / 256 * 256;
      J.chunk = (uint32_t)chunk;
      J.nch = (uint32_t)((J.n + chunk - 1) / chunk);
    }
    J.digit_base = (uint32_t)p.ndigits;
    J.bucket_base = (uint32_t)p.nbt;
    J.hist_base = (uint32_t)p.nh;
    J.plane_base = (uint32_t)p.nplanes;
    // about two bucket additions per quad (four lanes) before each block's tree
    J.bpb = std::max<uint32_t>(1, J.nb / 2 / (BP_THREADS / 2));
    J.blk_digits = (uint32_t)p.digit_blocks;
    J.blk_hs = (uint32_t)p.hs_blocks;
    p.ndigits += (uint64_t)J.nw * J.n;
    p.nbt += (uint64_t)J.nwb * J.nb;
    p.nh += (uint64_t)J.nwb * J.nb * J.nch;
    p.nplanes += (uint64_t)J.nwb * J.c;
    p.digit_blocks += J.digits_pw ? cdiv((uint64_t)J.n * J.nw, 256) : cdiv(J.n, 256);
    p.hs_blocks += J.pre ? (uint64_t)J.nch : (uint64_t)J.nw * J.nch;
    p.max_nb = std::max(p.max_nb, J.nb);
    p.max_nch = std::max(p.max_nch, J.nch);
    p.map.push_back(q);
    ZK_REQUIRE(p.ndigits < (1ull << 32) && p.nh < (1ull << 32) - 1 && p.nbt < (1ull << 31),
               "MSM batch too large for 32-bit offsets");
  }
  // the bucket reduction: grid sums of the large bucket sets after all the
  // buckets, then the reduction table in job order
  for (JobDev& J : p.jobs) {
    J.grid_lg = J.grid_base = 0;
    J.blk_gs = (uint32_t)p.gs_blocks;
    if (J.nb >= GRID_MIN_NB) {
      J.grid_lg = (uint32_t)(J.c - 1) / 2;
      const uint32_t L = 1u << J.grid_lg, R = J.nb >> J.grid_lg;
      J.grid_base = (uint32_t)(p.nbt + p.ngrid);
      p.ngrid += (uint64_t)J.nwb * (L + R);
      p.gs_blocks += (uint64_t)J.nwb * (L - 1 + R);
      // quads of about two entries each (R >= L entries at most per sum)
      while (p.gs_threads < (uint32_t)BP_THREADS && p.gs_threads < 2 * R) p.gs_threads *= 2;
    }
  }
  ZK_REQUIRE(p.nbt + p.ngrid < (1ull << 31), "MSM batch too large for 32-bit offsets");
  for (const JobDev& J : p.jobs) {
    JobDev e = J;
    e.pstride = (uint32_t)J.c;
    if (!J.grid_lg) {
      e.set_stride = J.nb;
      e.lg = (uint32_t)J.c - 1;
      e.poff = 0;
      e.blk_bp = (uint32_t)p.bp_blocks;
      p.bp_blocks += (uint64_t)J.nwb * J.c * J.bpb;
      p.red.push_back(e);
      continue;
    }
    const uint32_t L = 1u << J.grid_lg, R = J.nb >> J.grid_lg;
    e.set_stride = L + R;
    e.bpb = 1;  // L, R <= 128: one block per plane
    // column sums: digit values l in [1, L), planes 0 .. grid_lg - 1
    e.bucket_base = J.grid_base;
    e.nb = L;
    e.lg = J.grid_lg;
    e.c = (int)J.grid_lg;
    e.poff = 0;
    e.blk_bp = (uint32_t)p.bp_blocks;
    p.bp_blocks += (uint64_t)J.nwb * e.c;
    p.red.push_back(e);
    // row sums: digit values r in [1, R], planes grid_lg .. c - 1
    e.bucket_base = J.grid_base + L;
    e.nb = R;
    e.lg = (uint32_t)J.c - 1 - J.grid_lg;
    e.c = (int)e.lg + 1;
    e.poff = J.grid_lg;
    e.blk_bp = (uint32_t)p.bp_blocks;
    p.bp_blocks += (uint64_t)J.nwb * e.c;
    p.red.push_back(e);
  }
  const uint64_t E = p.ndigits;  // bound on the bucket entries
  // thread tasks: enough of them to fill the device, long enough to amortize
  bool tuned = true;
  for (int q = 0; q < njobs; q++) tuned = tuned && in[q].use_tuning;
  const int kd = E && tuned ? tuning().msm_kdiv_log[std::min(33, floor_log2(E))].load() : 0;
  p.K = (uint32_t)std::max<uint64_t>(4, std::min<uint64_t>(E >> (kd > 0 ? kd : 17), 64));
  // With few buckets and few entries in all (a small MSM, or full-width row
  // terms over precomputed windows) the device has room for a wavefront per bucket, and
  // a tree's depth beats a thread's chain of dependent additions: buckets of
  // 32 entries or more become wavefront tasks, and buckets with more than
  // FIN_THREAD_MIN partial sums are finished by a wavefront tree.
  const bool few_buckets = p.nbt <= FEW_BUCKETS && E <= FEW_ENTRIES;
  // otherwise wavefront tasks only for buckets far above the typical size (a
  // window's few possible top digits, or small-integer scalars piling into few
  // buckets): at least 32 tasks' worth and four times the average bucket
  const uint64_t avg_bucket = p.nbt ? E / p.nbt : 0;
  p.large = few_buckets ? 32u
                        : (uint32_t)std::min<uint64_t>(
                              1u << 30, std::max<uint64_t>({128, 32 * (uint64_t)p.K, 4 * avg_bucket}));
  // With few buckets and entries in all the batch is bound by chains of dependent
  // additions, not by throughput: additions in the wavefront tasks and the
  // finalize step are done by quads of lanes (shorter chains per point
  // operation), and wavefront tasks are shorter.
  p.quad = p.nbt <= 4 * FEW_BUCKETS && E <= FEW_ENTRIES;
  p.wg_entries = p.quad ? WG_TASK_ENTRIES_QUAD : WG_TASK_ENTRIES;
  p.max_th_tasks = E / p.K + p.nbt;
  // a large bucket of c entries makes ceil(c / WG_TASK_ENTRIES) tasks, and at
  // most E / large buckets are large
  p.max_wg_tasks = E / p.wg_entries + E / p.large + 1;
  p.max_partials = p.max_th_tasks + p.max_wg_tasks;
  // a thread per bucket unless a bucket holds several times the average
  // number of partial sums (a tree over a wavefront costs ~7 dependent
  // additions, so only far-above-average buckets gain from it)
  const uint64_t avg = p.nbt ? (E / p.K + p.nbt - 1) / p.nbt : 1;
  p.fin_max = few_buckets ? (uint32_t)FIN_THREAD_MIN : (uint32_t)std::max<uint64_t>(FIN_THREAD_MIN, 4 * avg);
  // short thread tasks leave many partial sums per bucket: a small tree per
  // bucket keeps the finalize chain short
  p.fin_group = 1;
  // The finalize step is a chain of dependent additions per bucket; with few
  // enough buckets that quads of lanes (up to about one wavefront per SIMD)
  // can share them, cooperative additions shorten the chains ~3x.
  p.fin_quad = p.quad || p.nbt <= FIN_QUAD_BUCKETS;
  if (p.fin_quad) {  // quads of about two partial sums each
    uint32_t quads = 1;
    while (quads < 16 && 2 * quads < avg && 8 * quads * p.nbt <= FIN_QUAD_LANES) quads *= 2;
    p.fin_group = 4 * quads;
  } else {
    while (p.fin_group < 64 && 4 * p.fin_group < avg) p.fin_group *= 2;
  }
  return p;
}

// The buffers of one batch, in a fixed order of workspace requests (every
// request is made before the first launch, so a workspace in arena mode can
// be sized by replaying the requests without launching anything).
struct MsmBufs {
  uint32_t *digits, *hist, *cnt, *off, *nt, *part_off, *sorted, *part, *buckets, *win, *bp_part, *heavy, *meta,
      *win_host;
  uint4 *th_tasks, *wg_tasks;
  JobDev *jt_host, *jt_dev, *rt_host, *rt_dev;
};

static MsmBufs msm_buffers(const BatchPlan& p, Workspace& ws, int XW) {
  const size_t nj = p.jobs.size();
  MsmBufs b;
  b.digits = ws.get(S_DIGITS, p.ndigits * 4);
  b.hist = ws.get(S_COUNTS, p.nh * 4);
  b.cnt = ws.get(S_CNT_A, p.nbt * 4);
  b.off = ws.get(S_OFF_A, p.nbt * 4);
  b.nt = ws.get(S_CNT_B, p.nbt * 4);
  b.part_off = ws.get(S_OFF_B, p.nbt * 4);
  b.sorted = ws.get(S_SORTED, p.ndigits * 4);
  b.th_tasks = ws.get<uint4>(S_TASKS, p.max_th_tasks * 16);
  b.wg_tasks = ws.get<uint4>(S_PART1, p.max_wg_tasks * 16);
  b.part = ws.get(S_PART0, p.max_partials * XW * 4);
  b.buckets = ws.get(S_SEG, (p.nbt + p.ngrid) * XW * 4);
  // plane sums: written by the kernels straight into pinned host memory when
  // the workspace's host buffers are device-visible, else copied back
  b.win = ws.host_mapped() ? nullptr : ws.get(S_WIN, p.nplanes * XW * 4);
  b.bp_part = ws.get(S_BP_PART, p.bp_blocks * XW * 4);
  b.heavy = ws.get(S_HEAVY, p.nbt * 4);
  b.meta = ws.get(S_META, 64 * 4);  // [2] partials [3] entries [8..10] thread tasks, wavefront tasks, heavy buckets
  b.win_host = ws.host<uint32_t>(S_WIN, p.nplanes * XW * 4);
  ws.get(S_SCRATCH, (size_t)cdiv(p.nbt, 2048) * 4 + 64);
  // a job table beyond the kernel arguments, through pinned memory (the
  // workspace is not reused before this stream has completed)
  b.jt_host = b.jt_dev = b.rt_host = b.rt_dev = nullptr;
  if (nj > (size_t)INLINE_JOBS) {
    b.jt_host = ws.host<JobDev>(S_JOBS, nj * sizeof(JobDev));
    b.jt_dev = ws.get<JobDev>(S_JOBS, nj * sizeof(JobDev));
  }
  const size_t nr = p.red.size();
  if (nr > (size_t)INLINE_JOBS) {
    b.rt_host = ws.host<JobDev>(S_RED, nr * sizeof(JobDev));
    b.rt_dev = ws.get<JobDev>(S_RED, nr * sizeof(JobDev));
  }
  return b;
}

void msm_arena_need(const MsmInput* in, int njobs, int group, size_t* dev_bytes, size_t* host_bytes) {
  const BatchPlan p = batch_plan(in, njobs, group == 1 ? 0 : 1);
  Workspace count;
  count.set_arena(nullptr, SIZE_MAX, nullptr, SIZE_MAX);
  if (!p.jobs.empty()) msm_buffers(p, count, group == 1 ? PointIO<Fq>::XYZZ_WORDS : PointIO<Fq2>::XYZZ_WORDS);
  *dev_bytes = count.arena_dev_used();
  *host_bytes = count.arena_host_used();
}

template <class F>
void msm_enqueue_batch(const MsmInput* in, int njobs, Workspace& ws, hipStream_t st, MsmPending* pend, int prio) {
  constexpr int XW = PointIO<F>::XYZZ_WORDS;
  ZK_REQUIRE(njobs >= 0, "negative MSM count");
  for (int q = 0; q < njobs; q++) {
    pend[q] = MsmPending();
    pend[q].xyzz_words = XW;
  }
  const BatchPlan p = batch_plan(in, njobs, PointIO<F>::AFF_WORDS == 16 ? 0 : 1);
  const int nj = (int)p.jobs.size();
  if (nj == 0) return;
  const uint32_t nbt = (uint32_t)p.nbt;
  const bool g1 = PointIO<F>::AFF_WORDS == 16;

  // all buffers first (a buffer that grows is replaced by a new one)
  const MsmBufs bf = msm_buffers(p, ws, XW);
  uint32_t *digits = bf.digits, *hist = bf.hist, *cnt = bf.cnt, *off = bf.off, *nt = bf.nt,
           *part_off = bf.part_off, *sorted = bf.sorted, *part = bf.part, *buckets = bf.buckets, *win = bf.win,
           *bp_part = bf.bp_part, *heavy = bf.heavy, *meta = bf.meta, *win_host = bf.win_host;
  uint4 *th_tasks = bf.th_tasks, *wg_tasks = bf.wg_tasks;
  auto table = [&](const std::vector<JobDev>& v, JobDev* th, JobDev* td) {
    BatchDev t{};
    t.njobs = (int)v.size();
    t.prio = prio;
    if (v.size() <= (size_t)INLINE_JOBS) {
      for (size_t k = 0; k < v.size(); k++) t.inl[k] = v[k];
    } else {
      std::memcpy(th, v.data(), v.size() * sizeof(JobDev));
      ZK_HIP(hipMemcpyAsync(td, th, v.size() * sizeof(JobDev), hipMemcpyHostToDevice, st));
      t.jobs = td;
    }
    return t;
  };
  const BatchDev dev = table(p.jobs, bf.jt_host, bf.jt_dev);
  const BatchDev red = table(p.red, bf.rt_host, bf.rt_dev);
  for (int k = 0; k < nj; k++) {
    MsmPending& pd = pend[p.map[k]];
    pd.empty = false;
    pd.c = p.jobs[k].c;
    pd.nw = (int)p.jobs[k].nwb;
    pd.win_host = win_host + (size_t)p.jobs[k].plane_base * XW;
  }
  uint32_t* const win_out = win ? win : win_host;
  const size_t lds = (size_t)p.max_nb * 4;
  {
    ProfScope ps(g1 ? "msm_digits_g1" : "msm_digits_g2", st, (double)p.ndigits);
    hipLaunchKernelGGL(k_msm_digits<F>, dim3((unsigned)p.digit_blocks), dim3(256), 0, st, dev, digits);
    ZK_HIP(hipGetLastError());
  }
  {
    ProfScope ps("msm_sort", st, (double)p.ndigits);
    hipLaunchKernelGGL(k_msm_hist, dim3((unsigned)p.hs_blocks), dim3(HS_THREADS), lds, st, dev, digits, hist);
    ZK_HIP(hipGetLastError());
    // bucket sizes and task counts, then the buckets' first slots and first partial sums
    // lanes per bucket: about 16 histogram rows each, at most 8 (a wavefront's
    // load then reads 8 consecutive buckets of 8 rows; 16 lanes measured 3%
    // slower on the proof, 4 lanes 1.5%)
    uint32_t lg_group = 2;
    while (lg_group < 3 && p.max_nch > (16u << lg_group)) lg_group++;
    hipLaunchKernelGGL(k_msm_colscan, dim3(cdiv((uint64_t)nbt << lg_group, 256)), dim3(256), 0, st, dev, hist, nbt,
                       p.K, p.large, p.wg_entries, cnt, nt, meta + 8, lg_group);
    ZK_HIP(hipGetLastError());
    scan_exclusive2(cnt, off, meta + 3, nt, part_off, meta + 2, nbt, ws, S_SCRATCH, st);
    hipLaunchKernelGGL(k_msm_scatter, dim3((unsigned)p.hs_blocks), dim3(HS_THREADS), lds, st, dev, digits, hist, off,
                       sorted);
    ZK_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_msm_make_tasks, dim3(cdiv(nbt, 256)), dim3(256), 0, st, dev, cnt, off, part_off, nbt, p.K,
                     p.large, p.wg_entries, p.fin_max, meta + 8, th_tasks, wg_tasks, heavy);
  ZK_HIP(hipGetLastError());
  {
    ProfScope ps(g1 ? "msm_acc_points_g1" : "msm_acc_points_g2", st, -1.0, true);
    hipEvent_t e0, e1;
    ps.bind_events(&e0, &e1);
    // capped grids with stride loops: the task counts are only known on the device
    const unsigned th_blocks = (unsigned)std::min<uint64_t>(cdiv(p.max_th_tasks, 64), 65536);
    const unsigned wg_blocks = (unsigned)std::min<uint64_t>(p.max_wg_tasks, 4096);
    launch_ev(e0, e1, k_msm_acc<F>, dim3(th_blocks + wg_blocks), dim3(64), 0, st, dev, th_tasks, wg_tasks,
              meta + 8, th_blocks, sorted, part, p.quad ? 1 : 0, meta + 3, ps.work_word());
    ZK_HIP(hipGetLastError());
  }
  {
    ProfScope ps(g1 ? "msm_finalize_g1" : "msm_finalize_g2", st, (double)nbt);
    const unsigned light_blocks = cdiv(nbt, 64 / p.fin_group);
    const unsigned heavy_blocks = (unsigned)std::min<uint64_t>(nbt, 1024);
    hipLaunchKernelGGL(k_msm_finalize<F>, dim3(light_blocks + heavy_blocks), dim3(64), 0, st, nt, part_off, part, nbt,
                       meta + 8, heavy, light_blocks, p.fin_max, p.fin_group, p.fin_quad ? 1 : 0, buckets, prio);
    ZK_HIP(hipGetLastError());
  }
  if (p.gs_blocks) {
    double adds = 0;  // about one addition per bucket for the rows and one for the columns
    for (const JobDev& J : p.jobs)
      if (J.grid_lg) adds += 2.0 * J.nwb * J.nb;
    ProfScope ps(g1 ? "msm_gridsums_g1" : "msm_gridsums_g2", st, adds);
    hipLaunchKernelGGL(k_msm_gridsums<F>, dim3((unsigned)p.gs_blocks), dim3(p.gs_threads), 0, st, dev, buckets);
    ZK_HIP(hipGetLastError());
  }
  {
    double adds = 0;
    for (const JobDev& e : p.red) adds += (double)e.nwb * e.c * e.nb / 2;
    ProfScope ps(g1 ? "msm_bitplanes_g1" : "msm_bitplanes_g2", st, adds);
    uint32_t per_block = 1;
    for (const JobDev& e : p.red) per_block = std::max(per_block, (e.nb / 2 + e.bpb - 1) / e.bpb);
    // quads of about two bucket additions each: 2 per_block lanes (64 to BP_THREADS)
    unsigned bp_threads = 64;
    while (bp_threads < (unsigned)BP_THREADS && bp_threads < 2 * per_block) bp_threads *= 2;
    hipLaunchKernelGGL(k_msm_bitplanes<F>, dim3((unsigned)p.bp_blocks), dim3(bp_threads), 0, st, red, buckets,
                       bp_part, win_out);
    ZK_HIP(hipGetLastError());
    // planes of one block each are final already
    bool split = false;
    for (const JobDev& e : p.red) split = split || e.bpb > 1;
    if (split) {
      hipLaunchKernelGGL(k_msm_plane_sums<F>, dim3((unsigned)p.nplanes), dim3(64), 0, st, red, bp_part, win_out);
      ZK_HIP(hipGetLastError());
    }
  }
  if (win) ZK_HIP(hipMemcpyAsync(win_host, win, p.nplanes * XW * 4, hipMemcpyDeviceToHost, st));
}

// Horner over the bit planes on the host; call after the MSM's stream has completed.
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
  msm_enqueue_batch<F>(&in, 1, ws, st, &pend, 0);
  ZK_HIP(hipStreamSynchronize(st));
  return msm_finish<F>(pend);
}

void msm_enqueue_batch_g1(const MsmInput* in, int njobs, Workspace& ws, hipStream_t st, MsmPending* pend, int prio) {
  msm_enqueue_batch<Fq>(in, njobs, ws, st, pend, prio);
}
void msm_enqueue_batch_g2(const MsmInput* in, int njobs, Workspace& ws, hipStream_t st, MsmPending* pend, int prio) {
  msm_enqueue_batch<Fq2>(in, njobs, ws, st, pend, prio);
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
    if (!F::cis_zero(z)) acc = F::mul(acc, z);
  }
  F inv = F::inv(acc);
  for (uint32_t jj = j1; jj > j0; jj--) {
    const uint32_t j = jj - 1;
    const uint32_t* p = xyzz + (size_t)j * XW;
    const F z = F::load(p + 3 * CW);
    Affine<F> a;
    if (F::cis_zero(z)) {
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
