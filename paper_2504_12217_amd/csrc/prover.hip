// Groth16 setup and prove for Y = X W (Section II: Gen and Prove; Section III:
// the circuits).  The constraint systems are never materialized: every
// quantity the protocol needs is a closed-form function of the shape, the
// circuit kind and the inputs.
//
// Domain and rows.  Row c of the constraint system sits at omega^c of the
// domain H of size N = 2^L >= m + l + 1: the m multiplication rows, then one
// input-consistency row per public variable t <= l (A = variable t, B = C = 0),
// then zero rows.  L_c is the Lagrange basis of H.
//
// Variables.  0 = constant 1; x_ik at 1 + i n + k; y_ij at 1 + a n + i b + j;
// w_kj at l + 1 + k b + j; then the auxiliary variables of each kind:
//   PLAIN      p_ijk = x_ik w_kj (k < n-1); row (i b + j) n + k:
//              x_ik * w_kj = p_ijk, last row = y_ij - sum_k p_ijk
//   PLAIN_ADD  p_ijk for every k; rows (i b + j)(n+1) + k: x_ik * w_kj = p_ijk,
//              then (sum_k p_ijk) * 1 = y_ij
//   PLAIN_PSQ  prefix sums s_ijk (k < n-1); row (i b + j) n + k:
//              x_ik * w_kj = s_ijk - s_ij(k-1), last row = y_ij - s_ij(n-2)
//   CRPC_PSQ   prefix sums s_k of X_k(z) W_k(z) (k < n-1); row k:
//              X_k(z) * W_k(z) = s_k - s_(k-1), last row = Y(z) - s_(n-2)
//   CRPC       products P_k = X_k(z) W_k(z); rows k < n, then (sum_k P_k) * 1 = Y(z)
// with X_k(z) = sum_i z^(i b) x_ik, W_k(z) = sum_j z^j w_kj,
// Y(z) = sum_ij z^(i b + j) y_ij (Section III-A's identity at Z = z).
#include "prover.hpp"

#include <array>
#include <atomic>
#include <chrono>
#include <algorithm>
#include <thread>
#include <map>
#include <future>
#include <cstring>

#include "api_common.hpp"
#include "curve.hpp"
#include "field.hpp"
#include "msm.hpp"
#include "ntt.hpp"
#include "profile.hpp"
#include "tune.hpp"

namespace zkvc {

static int bitlen(uint64_t v) {
  int b = 0;
  while (v) {
    b++;
    v >>= 1;
  }
  return b;
}

bool kind_uses_z(uint32_t kind) { return kind == ZKVC_CRPC_PSQ || kind == ZKVC_CRPC; }

Layout r1cs_layout(uint32_t a, uint32_t n, uint32_t b, uint32_t kind) {
  Layout L;
  ZK_REQUIRE(a >= 1 && n >= 1 && b >= 1, "shape dimensions must be positive");
  ZK_REQUIRE(a <= 65535, "at most 65535 rows in X");  // the product kernel's grid rows
  ZK_REQUIRE(kind <= ZKVC_CRPC, "unknown circuit kind");
  ZK_REQUIRE((uint64_t)a * n * b <= (1ull << 28) && (uint64_t)n * 16384ull < (1ull << 40), "shape too large");
  L.a = a;
  L.n = n;
  L.b = b;
  L.kind = kind;
  L.ell = (uint64_t)a * n + (uint64_t)a * b;
  const uint64_t ab = (uint64_t)a * b;
  switch (kind) {
    case ZKVC_PLAIN: L.m = ab * n; L.naux = ab * (n - 1); L.aux_bits = 14; break;     // |x w| <= 2^14
    case ZKVC_PLAIN_ADD: L.m = ab * (n + 1); L.naux = ab * n; L.aux_bits = 14; break;
    case ZKVC_PLAIN_PSQ: L.m = ab * n; L.naux = ab * (n - 1); L.aux_bits = bitlen((uint64_t)(n > 1 ? n - 1 : 1) * 16384); break;
    case ZKVC_CRPC_PSQ: L.m = n; L.naux = n - 1; L.aux_bits = 253; break;
    default: L.m = n + 1; L.naux = n; L.aux_bits = 253; break;
  }
  L.y_bits = bitlen((uint64_t)n * 16384);
  L.w_start = L.ell + 1;
  L.aux_start = L.w_start + (uint64_t)n * b;
  L.nv = L.aux_start + L.naux;
  const uint64_t rows = L.m + L.ell + 1;
  L.log_n = 0;
  while ((1ull << L.log_n) < rows) L.log_n++;
  ZK_REQUIRE(L.log_n <= 28, "circuit needs a domain above 2^28");
  ZK_REQUIRE(L.nv < (1ull << 31), "too many variables");
  L.N = 1ull << L.log_n;
  const bool aux_in_a = kind == ZKVC_PLAIN_ADD || kind == ZKVC_CRPC;
  // G1 ranges with wide scalars store precomputed windows while all copies
  // stay within 256 MiB (the gathers then stay cache-friendly; larger tables
  // turn the random point reads into HBM and TLB misses)
  auto precompute = [](Seg& s) {
    const int max_copies = (int)std::min<uint64_t>(32, (256ull << 20) / (64ull * std::max<uint64_t>(s.count, 1)));
    int c = 0, nw = 1;
    if (max_copies >= 2) msm_choose_precomputed(s.count, s.bits, max_copies, &c, &nw);
    if (nw > 1) {
      s.pre_c = c;
      s.pre_nw = nw;
    }
  };
  auto push = [&](std::vector<Seg>& v, uint64_t start, uint64_t count, int bits, bool pre) {
    if (!count) return;
    Seg s;
    s.var_start = start;
    s.count = count;
    s.bits = bits;
    s.index = v.empty() ? 0 : v.back().index + v.back().count;
    s.point_offset = v.empty() ? 0 : v.back().point_offset + v.back().count * v.back().pre_nw;
    if (pre) precompute(s);
    v.push_back(s);
  };
  push(L.segA, 0, L.ell + 1, L.y_bits, true);
  if (aux_in_a) push(L.segA, L.aux_start, L.naux, L.aux_bits, true);
  push(L.segB, L.w_start, (uint64_t)n * b, 7, false);  // |w| <= 2^7
  if (aux_in_a) push(L.segB, 0, 1, 1, false);
  push(L.segL, L.w_start, (uint64_t)n * b, 7, true);
  push(L.segL, L.aux_start, L.naux, L.aux_bits, true);
  L.segH.count = L.N;  // h on the coset g H, one scalar per point
  L.segH.bits = 253;
  if (L.segH.count) precompute(L.segH);
  if (kind_uses_z(kind)) {
    // full-width row values W_k(z): always precomputed windows, so that the
    // host combines c plane sums instead of ~254
    Seg& R = L.segR;
    R.count = n;
    R.bits = 253;
    int c = 0, nw = 1;
    msm_choose_precomputed(n, R.bits, 32, &c, &nw);
    if (nw <= 1) {
      c = 8;
      nw = 32;
    }
    R.pre_c = c;
    R.pre_nw = nw;
  }
  return L;
}

// stored points of a query (every precomputed copy included)
static uint64_t seg_total(const std::vector<Seg>& v) {
  return v.empty() ? 0 : v.back().point_offset + v.back().count * v.back().pre_nw;
}

// ------------------------------------------------------------------ device helpers
// Canonical words of a small signed integer: v >= 0 -> v, v < 0 -> r - |v|.
__device__ __forceinline__ void encode_int(int64_t v, uint32_t w[8]) {
  if (v >= 0) {
    w[0] = (uint32_t)v;
    w[1] = (uint32_t)((uint64_t)v >> 32);
#pragma unroll
    for (int k = 2; k < 8; k++) w[k] = 0u;
    return;
  }
  const uint64_t mag = (uint64_t)(-v);
  uint64_t borrow = 0;
#pragma unroll
  for (int k = 0; k < 8; k++) {
    const uint64_t sub = k == 0 ? (mag & 0xffffffffull) : (k == 1 ? (mag >> 32) : 0ull);
    const uint64_t t = (uint64_t)FrParams::P32[k] - sub - borrow;
    w[k] = (uint32_t)t;
    borrow = (t >> 32) & 1u;
  }
}

__device__ __forceinline__ bool kind_uses_z_dev(uint32_t kind) { return kind == ZKVC_CRPC_PSQ || kind == ZKVC_CRPC; }

__device__ __forceinline__ void store_words(uint32_t* p, const uint32_t w[8]) {
  reinterpret_cast<uint4*>(p)[0] = make_uint4(w[0], w[1], w[2], w[3]);
  reinterpret_cast<uint4*>(p)[1] = make_uint4(w[4], w[5], w[6], w[7]);
}
__device__ __forceinline__ void store_int(uint32_t* p, int64_t v) {
  uint32_t w[8];
  encode_int(v, w);
  store_words(p, w);
}
__device__ __forceinline__ Fr fr_of_int(int64_t v) {
  uint32_t w[8];
  encode_int(v, w);
  return Fr::to_mont(Fr::unpack(w));
}
__device__ __forceinline__ void store_canonical(uint32_t* p, const Fr& x) { Fr::from_mont(x).store(p); }

// ------------------------------------------------------------------ setup kernels
constexpr int LG_CHUNK = 16;

// L_c(tau) = omega^c (tau^N - 1) / (N (tau - omega^c)), with Montgomery's
// simultaneous inversion over chunks of LG_CHUNK rows per thread.
__global__ void __launch_bounds__(128) k_lagrange(uint32_t N, int log_n, const uint32_t* consts, NttTables T,
                                                  uint32_t* Lc, uint32_t* prefix) {
  const uint32_t c0 = (blockIdx.x * blockDim.x + threadIdx.x) * LG_CHUNK;
  if (c0 >= N) return;
  const uint32_t c1 = c0 + LG_CHUNK < N ? c0 + LG_CHUNK : N;
  const Fr tau = Fr::load(consts);
  const Fr K = Fr::load(consts + 8);  // (tau^N - 1) / N
  const int sh = NTT_MAX_LOG - log_n;
  Fr acc = Fr::one();
  for (uint32_t c = c0; c < c1; c++) {
    const Fr d = Fr::sub(tau, pow_lookup(T.w[0], c << sh));
    acc.store(prefix + 8ull * c);
    d.store(Lc + 8ull * c);
    acc = Fr::mul(acc, d);
  }
  Fr inv = Fr::inv(acc);
  for (uint32_t cc = c1; cc > c0; cc--) {
    const uint32_t c = cc - 1;
    const Fr d = Fr::load(Lc + 8ull * c);
    const Fr dinv = Fr::mul(inv, Fr::load(prefix + 8ull * c));
    inv = Fr::mul(inv, d);
    Fr::mul(Fr::mul(pow_lookup(T.w[0], c << sh), K), dinv).store(Lc + 8ull * c);
  }
}

__global__ void k_zpow(const uint32_t* z, uint32_t count, uint32_t* out) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  const Fr base = Fr::load(z);
  Fr r = Fr::one();
  for (int bit = 31; bit >= 0; bit--) {
    r = Fr::sqr(r);
    if ((e >> bit) & 1u) r = Fr::mul(r, base);
  }
  r.store(out + 8ull * e);
}

struct VarParams {
  uint32_t kind, a, n, b;
  uint64_t ell, m, nv, w_start, aux_start;
  const uint32_t* L;
  const uint32_t* zpow;
  uint32_t *u, *v, *w;
};

// u_i(tau), v_i(tau), w_i(tau) for every variable: sums of L_c over the rows in
// which the variable appears, weighted by its coefficient there.
__global__ void __launch_bounds__(128) k_var_polys(VarParams p) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.nv) return;
  auto Lc = [&](uint64_t c) { return Fr::load(p.L + 8ull * c); };
  auto zp = [&](uint64_t e) { return Fr::load(p.zpow + 8ull * e); };
  const uint32_t a = p.a, n = p.n, b = p.b, kind = p.kind;
  const bool crpc = kind == ZKVC_CRPC_PSQ || kind == ZKVC_CRPC;
  const uint64_t stride = kind == ZKVC_PLAIN_ADD ? n + 1 : n;  // rows per output in the plain family
  Fr U = Fr::zero(), V = Fr::zero(), W = Fr::zero();
  if (i <= p.ell) U = Lc(p.m + i);  // input-consistency row
  if (i == 0) {
    if (kind == ZKVC_PLAIN_ADD) {
      for (uint64_t ij = 0; ij < (uint64_t)a * b; ij++) V = Fr::add(V, Lc(ij * stride + n));
    } else if (kind == ZKVC_CRPC) {
      V = Lc(n);
    }
  } else if (i <= (uint64_t)a * n) {  // x_ik
    const uint64_t t = i - 1, ii = t / n, k = t % n;
    if (crpc) {
      U = Fr::add(U, Fr::mul(zp(ii * b), Lc(k)));
    } else {
      for (uint64_t j = 0; j < b; j++) U = Fr::add(U, Lc((ii * b + j) * stride + k));
    }
  } else if (i <= p.ell) {  // y_ij
    const uint64_t t = i - 1 - (uint64_t)a * n, ii = t / b, j = t % b;
    switch (kind) {
      case ZKVC_PLAIN: case ZKVC_PLAIN_PSQ: W = Lc((ii * b + j) * n + n - 1); break;
      case ZKVC_PLAIN_ADD: W = Lc((ii * b + j) * stride + n); break;
      case ZKVC_CRPC_PSQ: W = Fr::mul(zp(ii * b + j), Lc(n - 1)); break;
      default: W = Fr::mul(zp(ii * b + j), Lc(n)); break;
    }
  } else if (i < p.aux_start) {  // w_kj
    const uint64_t t = i - p.w_start, k = t / b, j = t % b;
    if (crpc) {
      V = Fr::mul(zp(j), Lc(k));
    } else {
      for (uint64_t ii = 0; ii < a; ii++) V = Fr::add(V, Lc((ii * b + j) * stride + k));
    }
  } else {  // auxiliary
    const uint64_t t = i - p.aux_start;
    switch (kind) {
      case ZKVC_PLAIN: {
        const uint64_t ij = t / (n - 1), k = t % (n - 1), base = ij * n;
        W = Fr::sub(Lc(base + k), Lc(base + n - 1));
        break;
      }
      case ZKVC_PLAIN_ADD: {
        const uint64_t ij = t / n, k = t % n, base = ij * stride;
        U = Lc(base + n);
        W = Lc(base + k);
        break;
      }
      case ZKVC_PLAIN_PSQ: {
        const uint64_t ij = t / (n - 1), k = t % (n - 1), base = ij * n;
        W = Fr::sub(Lc(base + k), Lc(base + k + 1));
        break;
      }
      case ZKVC_CRPC_PSQ: W = Fr::sub(Lc(t), Lc(t + 1)); break;
      default: U = Lc(n); W = Lc(t); break;
    }
  }
  U.store(p.u + 8ull * i);
  V.store(p.v + 8ull * i);
  W.store(p.w + 8ull * i);
}

// out_j = (beta u_i + alpha v_i + w_i) * f for i = start + j  (f = 1/delta or 1/gamma)
__global__ void k_lin(const uint32_t* u, const uint32_t* v, const uint32_t* w, uint64_t start, uint32_t count,
                      const uint32_t* consts, uint32_t* out) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= count) return;
  const Fr alpha = Fr::load(consts), beta = Fr::load(consts + 8), f = Fr::load(consts + 16);
  const uint64_t i = start + j;
  Fr s = Fr::add(Fr::add(Fr::mul(beta, Fr::load(u + 8ull * i)), Fr::mul(alpha, Fr::load(v + 8ull * i))),
                 Fr::load(w + 8ull * i));
  Fr::mul(s, f).store(out + 8ull * j);
}

// out_j = in_j * f (Montgomery form): the scalars of a precomputed window copy.
// out[k] = in[k stride] for k < n (Fr elements).
__global__ void k_gather_stride(const uint32_t* in, uint32_t stride, uint32_t n, uint32_t* out) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const uint4* src = reinterpret_cast<const uint4*>(in + 8ull * k * stride);
  uint4* dst = reinterpret_cast<uint4*>(out + 8ull * k);
  dst[0] = src[0];
  dst[1] = src[1];
}

__global__ void k_scale_fr(const uint32_t* in, uint32_t n, const uint32_t* f, uint32_t* out) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  Fr::mul(Fr::load(in + 8ull * j), Fr::load(f)).store(out + 8ull * j);
}

constexpr int H_CHUNK = 32;

// The H query in the Lagrange basis of the coset g H: the prover then needs
// h only as its values on the coset (the QAP quotient's pointwise step), not
// as coefficients, and the sum is the same group element
// sum_a h(x_a) [L_a(tau) Z(tau) / delta] = [h(tau) Z(tau) / delta].
// With x_a = g omega_N^a (the points of the coset transform, taken from the
// same tables), L_a(tau) = (tau^N - g^N) x_a / (N g^N (tau - x_a)), so
// scalar a = c x_a / (tau - x_a) for c = (tau^N - 1)(tau^N - g^N) / (delta N g^N).
// One thread per chunk of H_CHUNK scalars: the prefix products of the
// denominators go to `out` first, then one inversion gives every 1 / (tau - x_a)
// of the chunk (Montgomery's trick), which overwrites them.
__global__ void k_h_scalars(uint32_t count, int log_n, const uint32_t* consts, NttTables T, uint32_t* out) {
  const uint32_t j0 = (blockIdx.x * blockDim.x + threadIdx.x) * H_CHUNK;
  if (j0 >= count) return;
  const uint32_t j1 = j0 + H_CHUNK < count ? j0 + H_CHUNK : count;
  const Fr tau = Fr::load(consts), c = Fr::load(consts + 8), g = Fr::load(consts + 16);
  const int sh = NTT_MAX_LOG - log_n;
  auto point = [&](uint32_t j) { return Fr::mul(g, pow_lookup(T.w[0], j << sh)); };
  Fr acc = Fr::one();
  for (uint32_t j = j0; j < j1; j++) {
    acc.store(out + 8ull * j);  // product of the denominators before j
    acc = Fr::mul(acc, Fr::sub(tau, point(j)));
  }
  Fr inv = Fr::inv(acc);
  for (uint32_t jj = j1; jj > j0; jj--) {
    const uint32_t j = jj - 1;
    const Fr x = point(j);
    const Fr dinv = Fr::mul(inv, Fr::load(out + 8ull * j));
    inv = Fr::mul(inv, Fr::sub(tau, x));
    Fr::mul(Fr::mul(c, x), dinv).store(out + 8ull * j);
  }
}

// ------------------------------------------------------------------ prove kernels
// Y = X W in int32; block (i, j-tile): X row i is shared by the block.
// ---- witness kernels.  Each takes the proofs of a batch from a job table
// (blockIdx.z or blockIdx.y = proof); a single proof's job travels by value.
struct WitJob {
  uint32_t kind, a, n, b;
  uint64_t m, ell, aux_start, N;
  const int8_t* X;
  const int8_t* W;
  int32_t* Y;
  const uint32_t* zpow;
  uint32_t *assign, *aev, *bev, *cev;
  uint32_t *xk, *wk, *pkk, *yz;  // CRPC kinds: per-k sums and Y(z) partial sums
  uint32_t nyz;                  // number of Y(z) partial sums
  uint32_t* flag;                // pinned host word set when a row is not satisfied, or null
};
struct WitTable {
  const WitJob* jobs;  // device table, or null: use `one`
  WitJob one;
  __device__ __forceinline__ const WitJob& get(uint32_t q) const { return jobs ? jobs[q] : one; }
};


// A constraint row that the witness does not satisfy (A B != C): the rows
// whose three values are not a product by construction are checked, and the
// host reports an internal error instead of returning a proof that cannot
// verify.  Every writer stores the same value.
__device__ __forceinline__ void flag_unsatisfied(const WitJob& J) {
  if (J.flag) {
    *J.flag = 1u;
    __threadfence_system();
  }
}

// assignment (canonical words) of the constant, x, y and w variables

// Multiplication rows of the plain family, and their auxiliary variables.
__global__ void k_rows_plain(WitTable T) {
  const WitJob& J = T.get(blockIdx.y);
  const uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (kind_uses_z_dev(J.kind) || c >= J.m) return;
  const uint32_t n = J.n, b = J.b;
  const uint64_t stride = J.kind == ZKVC_PLAIN_ADD ? n + 1 : n;
  const uint64_t ij = c / stride, k = c % stride;
  const uint64_t i = ij / b, j = ij % b;
  auto x = [&](uint64_t kk) { return (int64_t)J.X[i * n + kk]; };
  auto w = [&](uint64_t kk) { return (int64_t)J.W[kk * b + j]; };
  if (J.kind == ZKVC_PLAIN_ADD && k == n) {  // (sum_k p_ijk) * 1 = y_ij
    int64_t sum = 0;
    for (uint64_t kk = 0; kk < n; kk++) sum += x(kk) * w(kk);
    if (sum != (int64_t)J.Y[ij]) flag_unsatisfied(J);
    store_int(J.aev + 8ull * c, sum);
    store_int(J.bev + 8ull * c, 1);
    store_int(J.cev + 8ull * c, J.Y[ij]);
    return;
  }
  const int64_t prod = x(k) * w(k);
  store_int(J.aev + 8ull * c, x(k));
  store_int(J.bev + 8ull * c, w(k));
  int64_t cval;
  switch (J.kind) {
    case ZKVC_PLAIN:
      if (k < n - 1) {
        cval = prod;
        store_int(J.assign + 8ull * (J.aux_start + ij * (n - 1) + k), prod);
      } else {  // y_ij - sum_{k' < n-1} p_ijk'
        int64_t s = 0;
        for (uint64_t kk = 0; kk + 1 < n; kk++) s += x(kk) * w(kk);
        cval = (int64_t)J.Y[ij] - s;
        if (cval != prod) flag_unsatisfied(J);
      }
      break;
    case ZKVC_PLAIN_ADD:
      cval = prod;
      store_int(J.assign + 8ull * (J.aux_start + ij * n + k), prod);
      break;
    default: {  // PLAIN_PSQ: s_k - s_(k-1), last row y - s_(n-2)
      int64_t before = 0;
      for (uint64_t kk = 0; kk < k; kk++) before += x(kk) * w(kk);
      if (k < n - 1) {
        store_int(J.assign + 8ull * (J.aux_start + ij * (n - 1) + k), before + prod);
        cval = (before + prod) - before;
      } else {
        cval = (int64_t)J.Y[ij] - before;
        if (cval != prod) flag_unsatisfied(J);
      }
      break;
    }
  }
  store_int(J.cev + 8ull * c, cval);
}

constexpr int RED_THREADS = 256;

constexpr int RED_WAVES = RED_THREADS / 64;

// Sum over a block of RED_THREADS lanes, valid in every lane: a butterfly
// over each wavefront's lanes (cross-lane reads, no barrier; every lane ends
// with the same canonical sum), then the wavefront sums through LDS.
__device__ Fr block_sum(Fr x, uint32_t* sh) {
  for (int o = 32; o >= 1; o >>= 1) {
    Fr y;
#pragma unroll
    for (int q = 0; q < NL; q++) y.v[q] = (uint32_t)__shfl_xor((int)x.v[q], o, 64);
    x = Fr::add(x, y);
  }
  const int wid = (int)(threadIdx.x >> 6);
  if ((threadIdx.x & 63u) == 0u) {
#pragma unroll
    for (int q = 0; q < NL; q++) sh[wid * NL + q] = x.v[q];
  }
  __syncthreads();
  Fr t = Fr::zero();
  for (int w = 0; w < RED_WAVES; w++) {
    Fr y;
#pragma unroll
    for (int q = 0; q < NL; q++) y.v[q] = sh[w * NL + q];
    t = Fr::add(t, y);
  }
  __syncthreads();  // sh is free again
  return t;
}

// Inclusive prefix sum over a block of RED_THREADS lanes (lane order): a
// shift-and-add scan inside each wavefront, then the sums of the wavefronts
// before this one through LDS.
__device__ Fr block_inclusive_scan(Fr x, uint32_t* sh) {
  const uint32_t lane = threadIdx.x & 63u;
  for (uint32_t o = 1; o < 64; o <<= 1) {
    Fr y;
#pragma unroll
    for (int q = 0; q < NL; q++) y.v[q] = (uint32_t)__shfl_up((int)x.v[q], o, 64);
    if (lane >= o) x = Fr::add(x, y);
  }
  const int wid = (int)(threadIdx.x >> 6);
  if (lane == 63u) {
#pragma unroll
    for (int q = 0; q < NL; q++) sh[wid * NL + q] = x.v[q];
  }
  __syncthreads();
  for (int w = 0; w < wid; w++) {
    Fr y;
#pragma unroll
    for (int q = 0; q < NL; q++) y.v[q] = sh[w * NL + q];
    x = Fr::add(x, y);
  }
  __syncthreads();  // sh is free again
  return x;
}

// Block k: X_k(z) = sum_i z^(i b) x_ik, W_k(z) = sum_j z^j w_kj and their product.
__device__ void crpc_xw_body(const WitJob& J, uint32_t k, uint32_t* sh) {
  const uint32_t a = J.a, n = J.n, b = J.b;
  Fr sx = Fr::zero(), sw = Fr::zero();
  for (uint32_t i = threadIdx.x; i < a; i += RED_THREADS)
    sx = Fr::add(sx, Fr::mul(Fr::load(J.zpow + 8ull * ((uint64_t)i * b)), fr_of_int(J.X[(size_t)i * n + k])));
  for (uint32_t j = threadIdx.x; j < b; j += RED_THREADS)
    sw = Fr::add(sw, Fr::mul(Fr::load(J.zpow + 8ull * j), fr_of_int(J.W[(size_t)k * b + j])));
  sx = block_sum(sx, sh);
  sw = block_sum(sw, sh);
  if (threadIdx.x == 0) {
    sx.store(J.xk + 8ull * k);
    sw.store(J.wk + 8ull * k);
    Fr::mul(sx, sw).store(J.pkk + 8ull * k);
  }
}

// Rows 0 .. m-1 and auxiliary variables of the CRPC kinds, one block per
// proof: the prefix sums s_k = sum_{k' <= k} P_k' come from a block-wide
// inclusive scan over chunks of RED_THREADS rows with a running carry.
__device__ void crpc_rows_body(const WitJob& J, uint32_t* sh, uint32_t* carry_sh) {
  const uint32_t kind = J.kind, n = J.n;
  const uint64_t aux_start = J.aux_start;
  const uint32_t *xk = J.xk, *wk = J.wk, *pk = J.pkk;
  uint32_t *assign = J.assign, *aev = J.aev, *bev = J.bev, *cev = J.cev;
  // Y(z) from the partial sums
  Fr yz = Fr::zero();
  for (uint32_t q = threadIdx.x; q < J.nyz; q += RED_THREADS) yz = Fr::add(yz, Fr::load(J.yz + 8ull * q));
  yz = block_sum(yz, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NL; q++) carry_sh[q] = yz.v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NL; q++) yz.v[q] = carry_sh[q];
  __syncthreads();
  Fr carry = Fr::zero();
  for (uint32_t k0 = 0; k0 < n; k0 += RED_THREADS) {
    const uint32_t k = k0 + threadIdx.x;
    const Fr P = k < n ? Fr::load(pk + 8ull * k) : Fr::zero();
    const Fr x = block_inclusive_scan(P, sh);  // over the chunk
    const Fr s = Fr::add(x, carry);  // s_k
    const Fr prev = Fr::sub(s, P);   // s_(k-1)
    if (k < n) {
      store_canonical(aev + 8ull * k, Fr::load(xk + 8ull * k));
      store_canonical(bev + 8ull * k, Fr::load(wk + 8ull * k));
      if (kind == ZKVC_CRPC) {
        store_canonical(cev + 8ull * k, P);
        store_canonical(assign + 8ull * (aux_start + k), P);
      } else if (k + 1 < n) {
        store_canonical(assign + 8ull * (aux_start + k), s);
        store_canonical(cev + 8ull * k, Fr::sub(s, prev));
      } else {
        store_canonical(cev + 8ull * k, Fr::sub(yz, prev));
      }
      // the last PSQ row (Y(z) - s_(n-2) = P_(n-1)) and the CRPC sum row
      // (s_(n-1) * 1 = Y(z)) both hold exactly when s_(n-1) = Y(z)
      if (k == n - 1 && !Fr::eq(s, yz)) flag_unsatisfied(J);
      if (kind == ZKVC_CRPC && k == n - 1) {  // (sum_k P_k) * 1 = Y(z)
        store_canonical(aev + 8ull * n, s);
        store_canonical(bev + 8ull * n, Fr::one());
        store_canonical(cev + 8ull * n, yz);
      }
    }
    // carry for the next chunk: the last thread's inclusive sum
    if (threadIdx.x == RED_THREADS - 1) {
#pragma unroll
      for (int q = 0; q < NL; q++) carry_sh[q] = s.v[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NL; q++) carry.v[q] = carry_sh[q];
    __syncthreads();
  }
}

// ---- the witness in two launches (a proving batch, or one proof)
// First: blocks below xw_blocks sum a CRPC proof's row k (crpc_xw_body); the others
// compute Y = X W, 256 entries of a row each, and (CRPC kinds) one partial
// sum of Y(z) = sum_ij z^(i b + j) y_ij per block into yz.
__global__ void __launch_bounds__(RED_THREADS) k_wit_first(WitTable T, uint32_t xw_blocks, uint32_t mm_bx) {
  __shared__ uint32_t sh[RED_THREADS * NL];
  const WitJob& J = T.get(blockIdx.y);
  if (blockIdx.x < xw_blocks) {
    if (!kind_uses_z_dev(J.kind) || blockIdx.x >= J.n) return;  // uniform per block
    crpc_xw_body(J, blockIdx.x, sh);
    return;
  }
  const uint32_t mm = blockIdx.x - xw_blocks;
  const uint32_t i = mm / mm_bx, bx = mm % mm_bx, j = bx * RED_THREADS + threadIdx.x;
  const uint32_t n = J.n, b = J.b;
  const bool in = i < J.a && j < b;
  // Y[i, the block's RED_THREADS columns]: each wavefront sums a quarter of
  // the k range and each lane four adjacent columns (one 32-bit load of W per
  // k when the rows are 4-byte aligned); the quarters meet in LDS.
  static_assert(RED_THREADS == 256, "four wavefronts of 64 lanes, four columns per lane");
  int32_t* part = reinterpret_cast<int32_t*>(sh);  // [4][RED_THREADS], before block_sum uses sh
  if (i < J.a) {  // uniform per block
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    const uint32_t k0 = (uint32_t)((uint64_t)n * wave / 4), k1 = (uint32_t)((uint64_t)n * (wave + 1) / 4);
    const uint32_t j0 = bx * RED_THREADS + 4u * lane;
    const int8_t* x = J.X + (size_t)i * n;
    int32_t acc[4] = {0, 0, 0, 0};
    if ((b & 3u) == 0 && (reinterpret_cast<uintptr_t>(J.W) & 3u) == 0) {
      if (j0 < b) {
        const int8_t* wp = J.W + j0;
#pragma unroll 8
        for (uint32_t k = k0; k < k1; k++) {
          const int32_t xv = x[k];
          const uint32_t w4 = *reinterpret_cast<const uint32_t*>(wp + (size_t)k * b);
#pragma unroll
          for (int q = 0; q < 4; q++) acc[q] += xv * (int32_t)(int8_t)(w4 >> (8 * q));
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < 4; q++)
        if (j0 + q < b)
          for (uint32_t k = k0; k < k1; k++) acc[q] += (int32_t)x[k] * (int32_t)J.W[(size_t)k * b + j0 + q];
    }
#pragma unroll
    for (int q = 0; q < 4; q++) part[wave * RED_THREADS + 4u * lane + q] = acc[q];
  }
  __syncthreads();
  int32_t y = 0;
  if (in) {
    y = part[threadIdx.x] + part[RED_THREADS + threadIdx.x] + part[2 * RED_THREADS + threadIdx.x] +
        part[3 * RED_THREADS + threadIdx.x];
    J.Y[(size_t)i * b + j] = y;
  }
  __syncthreads();  // part is read before block_sum reuses sh
  if (!kind_uses_z_dev(J.kind)) return;  // uniform per block
  Fr s = in ? Fr::mul(Fr::load(J.zpow + 8ull * ((uint64_t)i * b + j)), fr_of_int(y)) : Fr::zero();
  s = block_sum(s, sh);
  if (threadIdx.x == 0) s.store(J.yz + 8ull * mm);
}

// Second: block 0 forms a CRPC proof's rows (crpc_rows_body); the others write the
// public assignment (constant, x, y, w) and the rows from m on: rows m .. m
// + l take the public variable t = row - m in A, every later row is zero,
// and B, C are zero there (each value computed here, not read back).
__global__ void __launch_bounds__(RED_THREADS) k_wit_second(WitTable T) {
  __shared__ uint32_t sh[RED_THREADS * NL];
  __shared__ uint32_t carry_sh[NL];
  const WitJob& J = T.get(blockIdx.y);
  if (blockIdx.x == 0) {
    if (kind_uses_z_dev(J.kind)) crpc_rows_body(J, sh, carry_sh);  // uniform per block
    return;
  }
  const uint64_t e = (uint64_t)(blockIdx.x - 1) * blockDim.x + threadIdx.x;
  const uint64_t an = (uint64_t)J.a * J.n, ab = (uint64_t)J.a * J.b, nb = (uint64_t)J.n * J.b;
  auto value = [&](uint64_t i) -> int64_t {
    if (i == 0) return 1;
    if (i <= an) return J.X[i - 1];
    if (i <= an + ab) return J.Y[i - 1 - an];
    return J.W[i - 1 - an - ab];
  };
  if (e < 1 + an + ab + nb) store_int(J.assign + 8ull * e, value(e));
  const uint64_t c = J.m + e;
  if (c < J.N) {
    if (e <= J.ell)
      store_int(J.aev + 8ull * c, value(e));
    else
      store_int(J.aev + 8ull * c, 0);
    const uint4 z4 = make_uint4(0u, 0u, 0u, 0u);
    reinterpret_cast<uint4*>(J.bev + 8ull * c)[0] = z4;
    reinterpret_cast<uint4*>(J.bev + 8ull * c)[1] = z4;
    reinterpret_cast<uint4*>(J.cev + 8ull * c)[0] = z4;
    reinterpret_cast<uint4*>(J.cev + 8ull * c)[1] = z4;
  }
}

// The witness kernels for one proof outside a proving batch: Y, the
// assignment and the first `rows` rows of the evaluation vectors (rows <= m
// leaves out the input-consistency rows).  The CRPC kinds' per-k sums use
// workspace slots 230..233.
void enqueue_witness_one(const Layout& L, const uint32_t* zpow, uint64_t rows, const int8_t* X, const int8_t* W,
                         int32_t* Y, uint32_t* assign, uint32_t* aev, uint32_t* bev, uint32_t* cev, Workspace& ws,
                         hipStream_t st) {
  WitTable T{};
  WitJob& J = T.one;
  J.kind = L.kind;
  J.a = L.a;
  J.n = L.n;
  J.b = L.b;
  J.m = L.m;
  J.ell = L.ell;
  J.aux_start = L.aux_start;
  J.N = rows;
  J.X = X;
  J.W = W;
  J.Y = Y;
  J.zpow = zpow;
  J.assign = assign;
  J.aev = aev;
  J.bev = bev;
  J.cev = cev;
  const bool crpc = kind_uses_z(L.kind);
  J.xk = crpc ? ws.get(230, (size_t)L.n * 32) : nullptr;
  J.wk = crpc ? ws.get(231, (size_t)L.n * 32) : nullptr;
  J.pkk = crpc ? ws.get(232, (size_t)L.n * 32) : nullptr;
  const uint32_t mm_bx = cdiv(L.b, RED_THREADS), mm_blocks = mm_bx * L.a;
  J.yz = crpc ? ws.get(233, 32ull * mm_blocks) : nullptr;
  J.nyz = mm_blocks;
  J.flag = nullptr;
  const uint32_t xw_blocks = crpc ? L.n : 0u;
  hipLaunchKernelGGL(k_wit_first, dim3(xw_blocks + mm_blocks, 1), dim3(RED_THREADS), 0, st, T, xw_blocks, mm_bx);
  ZK_HIP(hipGetLastError());
  const uint64_t wide = std::max<uint64_t>(L.aux_start, rows > L.m ? rows - L.m : 0);
  hipLaunchKernelGGL(k_wit_second, dim3(1 + (unsigned)cdiv(wide, RED_THREADS), 1), dim3(RED_THREADS), 0, st, T);
  ZK_HIP(hipGetLastError());
  if (!crpc) {
    hipLaunchKernelGGL(k_rows_plain, dim3(cdiv(L.m, 256), 1), dim3(256), 0, st, T);
    ZK_HIP(hipGetLastError());
  }
}

size_t prove_footprint(const Layout& L) {
  const uint64_t scalars = L.ell + 1 + 2 * (uint64_t)L.n * L.b + L.naux + L.N;
  return (size_t)(32 * (L.nv + 3 * L.N) + 48 * scalars);
}

void enqueue_zpow(const uint32_t* z_dev, uint32_t count, uint32_t* out, hipStream_t st) {
  if (!count) return;
  hipLaunchKernelGGL(k_zpow, dim3(cdiv(count, 128)), dim3(128), 0, st, z_dev, count, out);
  ZK_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ host: setup
namespace {

void put_g1(std::vector<uint8_t>& out, const host::G1J& p) {
  zkvc_g1 g;
  g1_to_abi(p, &g);
  const uint8_t* b = reinterpret_cast<const uint8_t*>(&g);
  out.insert(out.end(), b, b + sizeof(g));
}
void put_g2(std::vector<uint8_t>& out, const host::G2J& p) {
  zkvc_g2 g;
  g2_to_abi(p, &g);
  const uint8_t* b = reinterpret_cast<const uint8_t*>(&g);
  out.insert(out.end(), b, b + sizeof(g));
}
template <class T>
void put_raw(std::vector<uint8_t>& out, const T& v) {
  const uint8_t* b = reinterpret_cast<const uint8_t*>(&v);
  out.insert(out.end(), b, b + sizeof(T));
}

host::G1J g1_gen() {
  const uint64_t x[4] = {1, 0, 0, 0}, y[4] = {2, 0, 0, 0};
  return host::G1J::from_affine(host::HFq::from_u64(x), host::HFq::from_u64(y));
}
host::G2J g2_gen() {
  host::HFq2 x{host::HFq::from_u64(G2Gen::X0), host::HFq::from_u64(G2Gen::X1)};
  host::HFq2 y{host::HFq::from_u64(G2Gen::Y0), host::HFq::from_u64(G2Gen::Y1)};
  return host::G2J::from_affine(x, y);
}
void scalar_words(const host::HFr& s, uint64_t w[4]) { s.to_u64(w); }

void upload_words(uint32_t* dst, const std::vector<uint32_t>& src, hipStream_t st) {
  ZK_HIP(hipMemcpyAsync(dst, src.data(), src.size() * 4, hipMemcpyHostToDevice, st));
  ZK_HIP(hipStreamSynchronize(st));
}

}  // namespace

zkvc_pk* groth16_setup(const Layout& L, const host::HFr toxic[5], const host::HFr* z, std::vector<uint8_t>& vk,
                       hipStream_t st) {
  using host::HFr;
  const HFr &tau = toxic[0], &alpha = toxic[1], &beta = toxic[2], &gamma = toxic[3], &delta = toxic[4];
  for (int k = 0; k < 5; k++) ZK_REQUIRE(!toxic[k].is_zero(), "toxic waste elements must be nonzero");
  const uint64_t Nexp[4] = {L.N, 0, 0, 0};
  const HFr tN = HFr::pow(tau, Nexp);
  ZK_REQUIRE(tN != HFr::one(), "tau lies in the evaluation domain");
  ZK_REQUIRE(tN != HFr::pow(HFr::from_uint(5), Nexp), "tau lies in the quotient's coset");
  const bool use_z = kind_uses_z(L.kind);
  if (use_z) ZK_REQUIRE(z != nullptr && !z->is_zero(), "this circuit kind needs a nonzero z");

  std::unique_ptr<zkvc_pk> pk(new zkvc_pk());
  static std::atomic<uint64_t> serial{0};
  pk->id = ++serial;
  pk->L = L;
  pk->device = current_device();
  pk->has_z = use_z;
  if (use_z) pk->z = *z;
  const NttTables& T = ntt_tables(pk->device);
  Workspace& ws = pk->ws;
  const uint64_t N = L.N, nv = L.nv;

  // constants (device Montgomery words)
  std::vector<uint32_t> consts(8 * 8, 0u);
  auto put = [&](int slot, const HFr& x) { x.to_dev(&consts[8 * slot]); };
  const HFr Ninv = HFr::inv(HFr::from_uint(L.N));
  put(0, tau);
  put(1, HFr::mul(HFr::sub(tN, HFr::one()), Ninv));
  uint32_t* dconsts = ws.get(1, consts.size() * 4);
  upload_words(dconsts, consts, st);

  uint32_t* Lc = ws.get(2, N * 32);
  uint32_t* prefix = ws.get(3, N * 32);
  {
    const size_t threads = cdiv(N, LG_CHUNK);
    hipLaunchKernelGGL(k_lagrange, dim3(cdiv(threads, 128)), dim3(128), 0, st, (uint32_t)N, L.log_n, dconsts, T, Lc,
                       prefix);
    ZK_HIP(hipGetLastError());
  }
  if (use_z) {
    const uint32_t cnt = L.a * L.b;
    pk->zpow.alloc((size_t)cnt * 32);
    std::vector<uint32_t> zw(8);
    z->to_dev(zw.data());
    uint32_t* dz = ws.get(4, 32);
    upload_words(dz, zw, st);
    hipLaunchKernelGGL(k_zpow, dim3(cdiv(cnt, 128)), dim3(128), 0, st, dz, cnt, pk->zpow.get());
    ZK_HIP(hipGetLastError());
  }
  uint32_t* u = ws.get(5, nv * 32);
  uint32_t* v = ws.get(6, nv * 32);
  uint32_t* w = ws.get(7, nv * 32);
  {
    VarParams vp{L.kind, L.a, L.n, L.b, L.ell, L.m, nv, L.w_start, L.aux_start, Lc,
                 use_z ? pk->zpow.get() : nullptr, u, v, w};
    hipLaunchKernelGGL(k_var_polys, dim3(cdiv(nv, 128)), dim3(128), 0, st, vp);
    ZK_HIP(hipGetLastError());
  }

  // A, B1, B2 queries straight from u and v
  const uint64_t nA = seg_total(L.segA), nB = seg_total(L.segB), nL = seg_total(L.segL);
  pk->qA.alloc(std::max<uint64_t>(nA, 1) * 64);
  pk->qB1.alloc(std::max<uint64_t>(nB, 1) * 64);
  pk->qB2.alloc(std::max<uint64_t>(nB, 1) * 128);
  pk->qL.alloc(std::max<uint64_t>(nL, 1) * 64);
  pk->qH.alloc(std::max<uint64_t>(L.segH.count * L.segH.pre_nw, 1) * 64);
  uint64_t maxseg = L.ell + 1;
  for (const Seg& s : L.segL) maxseg = std::max(maxseg, s.count);
  maxseg = std::max(maxseg, N);
  uint32_t* sc = ws.get(9, maxseg * 32);
  uint32_t* scaled = ws.get(12, maxseg * 32);
  // a G1 range and its precomputed copies: copy w from the scalars times 2^(c w)
  auto emit_g1 = [&](const uint32_t* sc_mont, const Seg& s, uint32_t* qbase) {
    fixed_base_g1(sc_mont, true, s.count, qbase + 16 * s.point_offset, false, ws, st);
    if (s.pre_nw <= 1) return;
    std::vector<uint32_t> fw(8 * s.pre_nw);
    const HFr step = HFr::pow(HFr::from_uint(2), std::array<uint64_t, 4>{(uint64_t)s.pre_c, 0, 0, 0}.data());
    HFr f = HFr::one();
    for (int w = 0; w < s.pre_nw; w++) {
      f.to_dev(&fw[8 * w]);
      f = HFr::mul(f, step);
    }
    uint32_t* dfw = ws.get(13, fw.size() * 4);
    upload_words(dfw, fw, st);
    for (int w = 1; w < s.pre_nw; w++) {
      hipLaunchKernelGGL(k_scale_fr, dim3(cdiv(s.count, 256)), dim3(256), 0, st, sc_mont, (uint32_t)s.count,
                         dfw + 8 * w, scaled);
      ZK_HIP(hipGetLastError());
      fixed_base_g1(scaled, true, s.count, qbase + 16 * (s.point_offset + (uint64_t)w * s.count), false, ws, st);
    }
  };
  for (const Seg& s : L.segA) emit_g1(u + 8 * s.var_start, s, pk->qA.get());
  for (const Seg& s : L.segB) {
    fixed_base_g1(v + 8 * s.var_start, true, s.count, pk->qB1.get() + 16 * s.point_offset, false, ws, st);
    fixed_base_g2(v + 8 * s.var_start, true, s.count, pk->qB2.get() + 32 * s.point_offset, false, ws, st);
  }
  // a G2 range's precomputed copies, as emit_g1
  auto emit_g2 = [&](const uint32_t* sc_mont, const Seg& s, uint32_t* qbase) {
    fixed_base_g2(sc_mont, true, s.count, qbase + 32 * s.point_offset, false, ws, st);
    std::vector<uint32_t> fw(8 * s.pre_nw);
    const HFr step = HFr::pow(HFr::from_uint(2), std::array<uint64_t, 4>{(uint64_t)s.pre_c, 0, 0, 0}.data());
    HFr f = HFr::one();
    for (int w = 0; w < s.pre_nw; w++) {
      f.to_dev(&fw[8 * w]);
      f = HFr::mul(f, step);
    }
    uint32_t* dfw = ws.get(13, fw.size() * 4);
    upload_words(dfw, fw, st);
    for (int w = 1; w < s.pre_nw; w++) {
      hipLaunchKernelGGL(k_scale_fr, dim3(cdiv(s.count, 256)), dim3(256), 0, st, sc_mont, (uint32_t)s.count,
                         dfw + 8 * w, scaled);
      ZK_HIP(hipGetLastError());
      fixed_base_g2(scaled, true, s.count, qbase + 32 * (s.point_offset + (uint64_t)w * s.count), false, ws, st);
    }
  };
  // row bases of the CRPC kinds: v_{w_k0}(tau) = L_k(tau) for B1 and B2
  uint32_t* rsc = nullptr;
  if (L.segR.count) {
    const Seg& R = L.segR;
    const size_t nr = (size_t)R.count * R.pre_nw;
    pk->qRB1.alloc(nr * 64);
    pk->qRB2.alloc(nr * 128);
    pk->qRL.alloc(nr * 64);
    rsc = ws.get(14, R.count * 32);
    hipLaunchKernelGGL(k_gather_stride, dim3(cdiv(R.count, 256)), dim3(256), 0, st, v + 8 * L.w_start, (uint32_t)L.b,
                       (uint32_t)R.count, rsc);
    ZK_HIP(hipGetLastError());
    emit_g1(rsc, R, pk->qRB1.get());
    emit_g2(rsc, R, pk->qRB2.get());
  }
  // L query: (beta u + alpha v + w) / delta over the witness variables
  std::vector<uint32_t> lc(8 * 3);
  alpha.to_dev(&lc[0]);
  beta.to_dev(&lc[8]);
  HFr::inv(delta).to_dev(&lc[16]);
  uint32_t* dlc = ws.get(8, lc.size() * 4);
  upload_words(dlc, lc, st);
  for (const Seg& s : L.segL) {
    hipLaunchKernelGGL(k_lin, dim3(cdiv(s.count, 128)), dim3(128), 0, st, u, v, w, s.var_start, (uint32_t)s.count,
                       dlc, sc);
    ZK_HIP(hipGetLastError());
    emit_g1(sc, s, pk->qL.get());
    if (rsc && s.var_start == L.w_start) {
      // row bases for L: the entries of w_k0, (alpha L_k(tau)) / delta
      hipLaunchKernelGGL(k_gather_stride, dim3(cdiv(L.segR.count, 256)), dim3(256), 0, st, sc, (uint32_t)L.b,
                         (uint32_t)L.segR.count, rsc);
      ZK_HIP(hipGetLastError());
      emit_g1(rsc, L.segR, pk->qRL.get());
    }
  }
  // H query: (tau^N - 1) / delta times the Lagrange basis of the coset g H at tau
  if (N > 1) {
    const HFr g = HFr::from_uint(5);  // the coset shift of the quotient's transforms
    const HFr gN = HFr::pow(g, Nexp);
    std::vector<uint32_t> hc(24);
    tau.to_dev(&hc[0]);
    HFr::mul(HFr::mul(HFr::sub(tN, HFr::one()), HFr::sub(tN, gN)), HFr::inv(HFr::mul(HFr::mul(delta, gN), HFr::from_uint(L.N))))
        .to_dev(&hc[8]);
    g.to_dev(&hc[16]);
    uint32_t* dhc = ws.get(10, hc.size() * 4);
    upload_words(dhc, hc, st);
    const uint32_t cnt = (uint32_t)N;
    hipLaunchKernelGGL(k_h_scalars, dim3(cdiv(cdiv(cnt, H_CHUNK), 128)), dim3(128), 0, st, cnt, (int)L.log_n, dhc, T,
                       sc);
    ZK_HIP(hipGetLastError());
    emit_g1(sc, L.segH, pk->qH.get());
  }
  // IC for the verification key: (beta u + alpha v + w) / gamma over 0..l
  HFr::inv(gamma).to_dev(&lc[16]);
  upload_words(dlc, lc, st);
  const uint64_t nic = L.ell + 1;
  hipLaunchKernelGGL(k_lin, dim3(cdiv(nic, 128)), dim3(128), 0, st, u, v, w, (uint64_t)0, (uint32_t)nic, dlc, sc);
  ZK_HIP(hipGetLastError());
  uint32_t* ic = ws.get(11, nic * 64);
  fixed_base_g1(sc, true, nic, ic, true, ws, st);
  std::vector<uint8_t> ic_host(nic * 64);
  ZK_HIP(hipMemcpyAsync(ic_host.data(), ic, ic_host.size(), hipMemcpyDeviceToHost, st));
  ZK_HIP(hipStreamSynchronize(st));

  // group constants on the host
  uint64_t e[4];
  const host::G1J g1 = g1_gen();
  const host::G2J g2 = g2_gen();
  scalar_words(alpha, e);
  pk->alpha1 = host::G1J::mul(g1, e);
  scalar_words(beta, e);
  pk->beta1 = host::G1J::mul(g1, e);
  pk->beta2 = host::G2J::mul(g2, e);
  scalar_words(delta, e);
  pk->delta1 = host::G1J::mul(g1, e);
  pk->delta2 = host::G2J::mul(g2, e);
  pk->delta1_table.build(pk->delta1);
  pk->delta2_table.build(pk->delta2);
  scalar_words(gamma, e);
  const host::G2J gamma2 = host::G2J::mul(g2, e);

  // verification key blob
  vk.clear();
  const char magic[8] = {'Z', 'K', 'V', 'C', '-', 'V', 'K', '1'};
  vk.insert(vk.end(), magic, magic + 8);
  const uint32_t hdr[6] = {1u, L.a, L.n, L.b, L.kind, (uint32_t)L.log_n};
  for (uint32_t h : hdr) put_raw(vk, h);
  uint32_t zw[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (use_z) z->to_u32(zw);
  for (uint32_t x : zw) put_raw(vk, x);
  put_g1(vk, pk->alpha1);
  put_g2(vk, pk->beta2);
  put_g2(vk, gamma2);
  put_g2(vk, pk->delta2);
  put_raw(vk, (uint64_t)nic);
  vk.insert(vk.end(), ic_host.begin(), ic_host.end());

  pk->key_bytes = pk->qA.size() + pk->qB1.size() + pk->qB2.size() + pk->qL.size() + pk->qH.size() + pk->zpow.size() +
                  pk->qRB1.size() + pk->qRB2.size() + pk->qRL.size();
  pk->ws.clear();  // setup scratch is not needed for proving
  return pk.release();
}

// ------------------------------------------------------------------ host: prove
namespace {
enum ProveSlot { P_ASSIGN = 20, P_AEV, P_BEV, P_CEV, P_XK, P_WK, P_PK, P_YZ };
enum SharedSlot { C_TABLE = 60, C_FLAG, C_XW, C_Y, C_WTAB };
// The H lane follows the quotient and ends the proof: its waves take
// instruction issue ahead of the G1 and G2 lanes' (results are unchanged).
constexpr int H_LANE_PRIO = 1;

// One MSM of a proof: a query segment (or the H query) and its scalars.
struct MsmJob {
  int group;  // 1 = G1, 2 = G2
  int query;  // ZKVC_Q_*
  MsmInput in;
};

// wk: for the CRPC kinds, W_k(z) = sum_j z^j w_kj for k < n (device Montgomery form).
std::vector<MsmJob> msm_jobs(const zkvc_pk* pk, const uint32_t* assign, const uint32_t* h_coset,
                             const uint32_t* wk) {
  const Layout& L = pk->L;
  std::vector<MsmJob> jobs;
  // In the CRPC kinds a variable w_kj enters one row only, the B side of
  // constraint k with coefficient z^j, so v_{w_kj} = z^j L_k and u, w vanish:
  // its B1, B2 and L key entries are z^j times those of w_k0 (setup makes
  // both from the same L_k).  Their n b terms sum to sum_k W_k(z) [entry of
  // w_k0]: n terms with the row values the witness already holds, over the
  // row bases stored with precomputed windows (the same group elements, so
  // the proof does not change).
  const bool collapse_w = kind_uses_z(L.kind) && wk != nullptr && L.segR.count == L.n;
  auto add = [&](int group, int query, const uint32_t* points, const Seg& s) {
    MsmJob j;
    j.group = group;
    j.query = query;
    j.in.points = points + (group == 1 ? 16 : 32) * s.point_offset;
    j.in.npoints = s.count;
    j.in.scalars = assign + 8 * s.var_start;
    j.in.nscalars = s.count;
    j.in.max_bits = s.bits;
    if (s.pre_nw > 1) {
      j.in.pre_c = s.pre_c;
      j.in.pre_nw = s.pre_nw;
    }
    if (collapse_w && s.var_start == L.w_start && s.count == (uint64_t)L.n * L.b) {
      const DevBuf& rb = query == ZKVC_Q_B2 ? pk->qRB2 : (query == ZKVC_Q_B1 ? pk->qRB1 : pk->qRL);
      j.in.points = rb.get();
      j.in.npoints = L.n;
      j.in.scalars = wk;
      j.in.nscalars = L.n;
      j.in.scalars_mont = true;
      j.in.max_bits = L.segR.bits;
      j.in.pre_c = L.segR.pre_c;
      j.in.pre_nw = L.segR.pre_nw;
    }
    jobs.push_back(j);
  };
  if (L.N > 1) {
    MsmJob j;
    j.group = 1;
    j.query = ZKVC_Q_H;
    j.in.points = pk->qH.get();
    j.in.npoints = L.N;
    j.in.scalars = h_coset;
    j.in.nscalars = L.N;
    j.in.scalars_mont = true;
    j.in.point_index_bitrev = 0;
    j.in.max_bits = L.segH.bits;
    if (L.segH.pre_nw > 1) {
      j.in.pre_c = L.segH.pre_c;
      j.in.pre_nw = L.segH.pre_nw;
    }
    jobs.push_back(j);
  }
  for (const Seg& s : L.segL) add(1, ZKVC_Q_L, pk->qL.get(), s);
  for (const Seg& s : L.segB) add(2, ZKVC_Q_B2, pk->qB2.get(), s);
  for (const Seg& s : L.segB) add(1, ZKVC_Q_B1, pk->qB1.get(), s);
  for (const Seg& s : L.segA) add(1, ZKVC_Q_A, pk->qA.get(), s);
  return jobs;
}

// Device buffers of one proof in flight.
struct Slot {
  uint32_t *assign, *aev, *bev, *cev;
  const uint32_t* wk;  // CRPC kinds: W_k(z) for k < n, else null
  int32_t* yh;      // pinned copy of Y
  int8_t *xh, *wh;  // pinned staging of X and W
};

// The copy of Y (all host-buffer jobs of a batch) back to pinned memory.
struct YCopy {
  void* dst = nullptr;
  const void* src = nullptr;
  size_t bytes = 0;
};

// Witness and evaluation vectors of every proof of a batch, one launch per
// kernel for all proofs.  X and W of all host-buffer proofs cross PCIe in one
// copy from pinned staging, and their Y comes back in one copy to pinned
// memory (described in *ycopy, enqueued by the caller); device-buffer proofs
// read and write the caller's buffers.  No host wait inside the enqueue.
// With bind (eager streams), the row event and end_ev are bound to the
// dispatch of the kernels they follow instead of recorded after them;
// otherwise the row event is recorded and end_ev is left to the caller.
std::vector<Slot> enqueue_witness_batch(const ProveJob* jobs, size_t nj, ProveGen& G, hipStream_t st, YCopy* ycopy,
                                        volatile uint32_t** flag_out, bool bind, hipEvent_t end_ev) {
  ZK_REQUIRE(nj <= 65535, "at most 65535 proofs per batch");
  // the row check writes straight into pinned host memory (cleared here; a
  // graph replay clears it before each launch)
  uint32_t* flag = G.shared.host<uint32_t>(C_FLAG, 4);
  *flag = 0u;
  *flag_out = flag;
  auto align = [](size_t v) { return (v + 255) & ~(size_t)255; };
  std::vector<size_t> xo(nj), wo(nj), yo(nj);
  size_t xw_bytes = 0, y_bytes = 0;
  for (size_t j = 0; j < nj; j++) {
    if (jobs[j].device_io) continue;
    const Layout& L = jobs[j].pk->L;
    xo[j] = xw_bytes;
    xw_bytes += align((size_t)L.a * L.n);
    wo[j] = xw_bytes;
    xw_bytes += align((size_t)L.n * L.b);
    yo[j] = y_bytes;
    y_bytes += align((size_t)L.a * L.b * 4);
  }
  int8_t* xw_host = xw_bytes ? G.shared.host<int8_t>(C_XW, xw_bytes) : nullptr;
  int8_t* xw_dev = xw_bytes ? G.shared.get<int8_t>(C_XW, xw_bytes) : nullptr;
  int8_t* y_host = y_bytes ? G.shared.host<int8_t>(C_Y, y_bytes) : nullptr;
  int8_t* y_dev = y_bytes ? G.shared.get<int8_t>(C_Y, y_bytes) : nullptr;
  std::vector<Slot> slots(nj);
  std::vector<WitJob> wj(nj);
  uint32_t max_a = 0, max_b = 0, max_n_crpc = 0;
  uint64_t max_pub = 0, max_m_plain = 0, max_tail = 0;
  bool any_crpc = false, any_plain = false;
  for (size_t j = 0; j < nj; j++) {
    const zkvc_pk* pk = jobs[j].pk;
    const Layout& L = pk->L;
    Workspace& ws = *G.slot_ws[j];
    Slot& S = slots[j];
    S.assign = ws.get(P_ASSIGN, L.nv * 32);
    S.aev = ws.get(P_AEV, L.N * 32);
    S.bev = ws.get(P_BEV, L.N * 32);
    S.cev = ws.get(P_CEV, L.N * 32);
    const bool dio = jobs[j].device_io;
    S.yh = dio ? nullptr : reinterpret_cast<int32_t*>(y_host + yo[j]);
    S.xh = dio ? nullptr : xw_host + xo[j];
    S.wh = dio ? nullptr : xw_host + wo[j];
    if (!dio) {
      std::memcpy(S.xh, jobs[j].X, (size_t)L.a * L.n);
      std::memcpy(S.wh, jobs[j].W, (size_t)L.n * L.b);
    }
    WitJob& J = wj[j];
    J.kind = L.kind;
    J.a = L.a;
    J.n = L.n;
    J.b = L.b;
    J.m = L.m;
    J.ell = L.ell;
    J.aux_start = L.aux_start;
    J.N = L.N;
    J.X = dio ? jobs[j].X : xw_dev + xo[j];
    J.W = dio ? jobs[j].W : xw_dev + wo[j];
    J.Y = dio ? jobs[j].Y : reinterpret_cast<int32_t*>(y_dev + yo[j]);
    J.zpow = pk->zpow.get();
    J.assign = S.assign;
    J.aev = S.aev;
    J.bev = S.bev;
    J.cev = S.cev;
    J.flag = flag;
    if (kind_uses_z(L.kind)) {
      J.xk = ws.get(P_XK, (size_t)L.n * 32);
      J.wk = ws.get(P_WK, (size_t)L.n * 32);
      S.wk = J.wk;
      J.pkk = ws.get(P_PK, (size_t)L.n * 32);
      J.yz = nullptr;  // sized below, by the batch's tiling of Y
      any_crpc = true;
      max_n_crpc = std::max(max_n_crpc, L.n);
    } else {
      J.xk = J.wk = J.pkk = J.yz = nullptr;
      S.wk = nullptr;
      any_plain = true;
      max_m_plain = std::max(max_m_plain, L.m);
    }
    max_a = std::max(max_a, L.a);
    max_b = std::max(max_b, L.b);
    max_pub = std::max<uint64_t>(max_pub, L.aux_start);
    max_tail = std::max<uint64_t>(max_tail, L.N - L.m);
  }
  if (xw_bytes) ZK_HIP(hipMemcpyAsync(xw_dev, xw_host, xw_bytes, hipMemcpyHostToDevice, st));
  // Y is computed RED_THREADS entries of a row per block, and each block of a
  // CRPC proof leaves one partial sum of Y(z)
  const uint32_t mm_bx = cdiv(max_b, RED_THREADS), mm_blocks = mm_bx * max_a;
  for (size_t j = 0; j < nj; j++) {
    if (!kind_uses_z(jobs[j].pk->L.kind)) continue;
    wj[j].yz = G.slot_ws[j]->get(P_YZ, 32ull * mm_blocks);
    wj[j].nyz = mm_blocks;
  }
  WitTable T{};
  if (nj == 1) {
    T.one = wj[0];
  } else {
    WitJob* th = G.shared.host<WitJob>(C_WTAB, nj * sizeof(WitJob));
    WitJob* td = G.shared.get<WitJob>(C_WTAB, nj * sizeof(WitJob));
    std::memcpy(th, wj.data(), nj * sizeof(WitJob));
    ZK_HIP(hipMemcpyAsync(td, th, nj * sizeof(WitJob), hipMemcpyHostToDevice, st));
    T.jobs = td;
  }
  const unsigned J = (unsigned)nj;
  // the CRPC row values first: when every proof is CRPC+PSQ they are all the
  // G2 lane needs (W_k(z) for the row terms; the CRPC kind's B query also
  // holds the constant, written with the public assignment), so it starts here
  bool rows_only = true;
  for (size_t j = 0; j < nj; j++) rows_only = rows_only && jobs[j].pk->L.kind == ZKVC_CRPC_PSQ;
  // the CRPC per-row sums and Y in one launch, then the CRPC rows and the
  // public assignment and tail rows in another
  const uint32_t xw_blocks = any_crpc ? max_n_crpc : 0u;
  const hipEvent_t row_bound = bind && rows_only ? G.wrow_ev : nullptr;
  launch_ev(nullptr, row_bound, k_wit_first, dim3(xw_blocks + mm_blocks, J), dim3(RED_THREADS), 0u, st, T, xw_blocks,
            mm_bx);
  ZK_HIP(hipGetLastError());
  if (rows_only && !bind) ZK_HIP(hipEventRecord(G.wrow_ev, st));
  const uint64_t wide = std::max<uint64_t>(max_pub, max_tail);
  const hipEvent_t end_bound = bind ? end_ev : nullptr;
  launch_ev(nullptr, any_plain ? nullptr : end_bound, k_wit_second, dim3(1 + (unsigned)cdiv(wide, RED_THREADS), J),
            dim3(RED_THREADS), 0u, st, T);
  ZK_HIP(hipGetLastError());
  if (any_plain) {
    launch_ev(nullptr, end_bound, k_rows_plain, dim3(cdiv(max_m_plain, 256), J), dim3(256), 0u, st, T);
    ZK_HIP(hipGetLastError());
  }
  if (!rows_only) ZK_HIP(hipEventRecord(G.wrow_ev, st));
  // Y of host-buffer jobs goes back after the quotients (off the path to the H lane)
  ycopy->dst = y_host;
  ycopy->src = y_dev;
  ycopy->bytes = y_bytes;
  return slots;
}

// A process-wide set of persistent host threads for the data-parallel host
// loops of a batch (plane combination and assembly per proof), so that no
// thread is created per batch.  Created on first use and never destroyed
// (its threads wait on a condition variable until the process ends).
class HostPool {
 public:
  explicit HostPool(size_t nthreads) {
    for (size_t t = 0; t < nthreads; t++)
      std::thread([this] {
        for (;;) {
          std::function<void()> task;
          {
            std::unique_lock<std::mutex> lock(mu_);
            cv_.wait(lock, [this] { return !queue_.empty(); });
            task = std::move(queue_.front());
            queue_.pop_front();
          }
          task();
        }
      }).detach();
  }
  void post(std::function<void()> fn) {
    {
      std::lock_guard<std::mutex> lock(mu_);
      queue_.push_back(std::move(fn));
    }
    cv_.notify_one();
  }

 private:
  std::deque<std::function<void()>> queue_;
  std::mutex mu_;
  std::condition_variable cv_;
};

size_t host_threads() {
  const unsigned hc = std::thread::hardware_concurrency();
  return hc ? std::min<size_t>(16, std::max<size_t>(1, hc / 2)) : 4;
}

HostPool& host_pool() {
  static HostPool* p = new HostPool(host_threads());
  return *p;
}

// Runs fn(i) for i < n on the calling thread plus up to threads - 1 helpers
// of the host pool.  Indices are claimed from a shared counter; the caller
// works too, so the call completes even if every helper is busy elsewhere,
// and it waits only for helpers that have started (a helper that starts
// after the loop has closed returns at once).  The first exception thrown by
// fn is rethrown on the calling thread after every started helper has
// stopped (indices not yet claimed are then skipped).
template <class Fn>
void parallel_for(size_t n, size_t threads, Fn&& fn) {
  threads = std::max<size_t>(1, std::min(threads, n));
  if (threads == 1) {
    for (size_t i = 0; i < n; i++) fn(i);
    return;
  }
  struct State {
    std::atomic<size_t> next{0};
    std::mutex mu;
    std::condition_variable cv;
    bool closed = false;
    int active = 0;
    std::exception_ptr err;
  };
  auto st = std::make_shared<State>();
  std::function<void(size_t)> body = [&fn](size_t i) { fn(i); };
  auto work = [st, n, &body] {
    try {
      for (size_t i; (i = st->next.fetch_add(1)) < n;) body(i);
    } catch (...) {
      st->next.store(n);
      std::lock_guard<std::mutex> lock(st->mu);
      if (!st->err) st->err = std::current_exception();
    }
  };
  for (size_t t = 1; t < threads; t++)
    host_pool().post([st, work] {
      {
        std::lock_guard<std::mutex> lock(st->mu);
        if (st->closed) return;
        st->active++;
      }
      work();
      std::lock_guard<std::mutex> lock(st->mu);
      if (--st->active == 0) st->cv.notify_all();
    });
  work();
  std::unique_lock<std::mutex> lock(st->mu);
  st->closed = true;
  st->cv.wait(lock, [&] { return st->active == 0; });
  if (st->err) std::rethrow_exception(st->err);
}

}  // namespace

TaskPool::TaskPool(int nthreads) {
  for (int t = 0; t < nthreads; t++)
    threads_.emplace_back([this] {
      for (;;) {
        std::packaged_task<void()> task;
        {
          std::unique_lock<std::mutex> lock(mu_);
          cv_.wait(lock, [this] { return stop_ || !queue_.empty(); });
          if (queue_.empty()) return;  // stopping with nothing left to run
          task = std::move(queue_.front());
          queue_.pop_front();
        }
        task();
      }
    });
}

TaskPool::~TaskPool() {
  {
    std::lock_guard<std::mutex> lock(mu_);
    stop_ = true;
  }
  cv_.notify_all();
  for (auto& t : threads_) t.join();
}

std::future<void> TaskPool::run(std::function<void()> fn) {
  std::packaged_task<void()> task(std::move(fn));
  std::future<void> f = task.get_future();
  {
    std::lock_guard<std::mutex> lock(mu_);
    queue_.push_back(std::move(task));
  }
  cv_.notify_one();
  return f;
}

// The lane streams every proving context of a device shares.  A process has
// few hardware queues (four by default) and a new stream takes the next one
// in turn: with lane streams per context, the lanes of every key created
// after the first landed on queues that the calling stream or other lanes
// already used, and those keys proved ~40% slower (0.92 against 0.67 ms per
// proof of [49,320]x[320,512]), their lanes serialized behind other work.
// Created on first use and kept for the process (released by the operating
// system at exit, never from a static destructor).  Contexts that prove
// concurrently from several host threads order their lane work on these
// streams; every wait is on an event recorded before it, so no cycle forms.
namespace {
struct SharedLanes {
  hipStream_t lanes[ProveCtx::LANES];
};
const SharedLanes& shared_lanes(int device) {
  static std::mutex mu;
  static std::map<int, SharedLanes*>* by_dev = new std::map<int, SharedLanes*>();
  std::lock_guard<std::mutex> lock(mu);
  auto it = by_dev->find(device);
  if (it != by_dev->end()) return *it->second;
  std::unique_ptr<SharedLanes> s(new SharedLanes());
  for (int lane = 0; lane < ProveCtx::LANES; lane++)
    ZK_HIP(hipStreamCreateWithFlags(&s->lanes[lane], hipStreamNonBlocking));
  SharedLanes* p = s.release();
  (*by_dev)[device] = p;
  return *p;
}
}  // namespace

ProveCtx::ProveCtx() {
  device = current_device();
  pool.reset(new TaskPool(4));
  const SharedLanes& sl = shared_lanes(device);
  for (int lane = 0; lane < LANES; lane++) lanes[lane] = sl.lanes[lane];
  ZK_HIP(hipStreamCreateWithFlags(&graph_stream, hipStreamNonBlocking));
  for (ProveGen& g : gen) {
    ZK_HIP(hipEventCreateWithFlags(&g.witness_ev, hipEventDisableTiming));
    ZK_HIP(hipEventCreate(&g.wrow_ev));  // may be bound to a kernel's dispatch
    ZK_HIP(hipEventCreateWithFlags(&g.quotient_ev, hipEventDisableTiming));
    ZK_HIP(hipEventCreateWithFlags(&g.fork_ev, hipEventDisableTiming));
    ZK_HIP(hipEventCreateWithFlags(&g.graph_ev, hipEventDisableTiming));
    for (int lane = 0; lane < LANES; lane++) {
      ZK_HIP(hipEventCreateWithFlags(&g.done_ev[lane], hipEventDisableTiming));
      ZK_HIP(hipEventCreateWithFlags(&g.join_ev[lane], hipEventDisableTiming));
      ZK_HIP(hipEventCreate(&g.lane_t[lane]));
    }
    for (auto& e : g.ev) ZK_HIP(hipEventCreate(&e));
  }
}

ProveCtx::~ProveCtx() {
  // wait for anything still queued on the lanes (the shared ones stay), then
  // release the context's own capture lanes
  for (int lane = 0; lane < LANES; lane++) {
    if (lanes[lane]) (void)hipStreamSynchronize(lanes[lane]);
    if (cap_lanes[lane]) {
      (void)hipStreamSynchronize(cap_lanes[lane]);
      (void)hipStreamDestroy(cap_lanes[lane]);
    }
  }
  if (graph_stream) {
    (void)hipStreamSynchronize(graph_stream);
    (void)hipStreamDestroy(graph_stream);
  }
  for (ProveGen& g : gen) {
    if (g.graph) (void)hipGraphExecDestroy(g.graph);
    release_graph_slots(g.graph_prof);
    if (g.fork_ev) (void)hipEventDestroy(g.fork_ev);
    if (g.graph_ev) (void)hipEventDestroy(g.graph_ev);
    if (g.witness_ev) (void)hipEventSynchronize(g.witness_ev), (void)hipEventDestroy(g.witness_ev);
    if (g.wrow_ev) (void)hipEventSynchronize(g.wrow_ev), (void)hipEventDestroy(g.wrow_ev);
    if (g.quotient_ev) (void)hipEventSynchronize(g.quotient_ev), (void)hipEventDestroy(g.quotient_ev);
    for (int lane = 0; lane < LANES; lane++) {
      if (g.done_ev[lane]) (void)hipEventDestroy(g.done_ev[lane]);
      if (g.join_ev[lane]) (void)hipEventDestroy(g.join_ev[lane]);
      if (g.lane_t[lane]) (void)hipEventDestroy(g.lane_t[lane]);
    }
    for (auto& e : g.ev)
      if (e) (void)hipEventDestroy(e);
  }
}

void ProveCtx::release_retired() {
  for (ProveGen& g : gen) {
    for (Workspace& w : g.lane_ws) w.release_retired();
    for (auto& w : g.slot_ws) w->release_retired();
    g.shared.release_retired();
  }
}

size_t ProveCtx::device_bytes() const {
  size_t s = 0;
  for (const ProveGen& g : gen) {
    for (const Workspace& w : g.lane_ws) s += w.bytes();
    for (const auto& w : g.slot_ws) s += w->bytes();
    s += g.shared.bytes();
  }
  return s;
}

size_t ProveCtx::host_bytes() const {
  size_t s = 0;
  for (const ProveGen& g : gen) {
    for (const Workspace& w : g.lane_ws) s += w.host_bytes();
    for (const auto& w : g.slot_ws) s += w->host_bytes();
    s += g.shared.host_bytes();
  }
  return s;
}

// Everything a begun batch needs to be finished.
struct BatchRun {
  ProveCtx* ctx = nullptr;
  int g = 0;
  bool finished = false;
  bool graphed = false;  // launched as a graph (records of its profiling scopes come from the graph)
  std::vector<ProveJob> jobs;
  std::vector<Slot> slots;
  std::vector<MsmInput> in_g1, in_g2, in_h;
  std::vector<int> own_g1, query_g1, own_g2, own_h;
  std::vector<MsmPending> pend_g1, pend_g2, pend_h;
  volatile uint32_t* flag_host = nullptr;  // pinned, written by the witness row check
  std::chrono::steady_clock::time_point host_t0;
  // the H MSMs on the quotient's own stream (no cross-stream wait between
  // them); a pipelined caller keeps them on the H lane so that its next
  // batch's witness need not wait behind them
  bool h_on_main = false;
};

void BatchRunDeleter::operator()(BatchRun* r) const { delete r; }

namespace {

// off by default: replaying a captured graph measured slower here than the
// eager multi-stream launches (the runtime dispatches a graph's nodes one by
// one in capture order, so the later lanes start later)
std::atomic<int> g_graphs{0};

// Stage and lane-end events: under capture they become event record nodes of
// the graph that each replay records (the host waits on them and times with them).
void record_ext(hipEvent_t e, hipStream_t st, bool capture) {
  if (capture)
    record_event(e, st);
  else
    ZK_HIP(hipEventRecord(e, st));
}

// Enqueues every device operation of a begun batch (eager, or under capture).
void enqueue_batch(ProveCtx& ctx, ProveGen& G, BatchRun& R, hipStream_t st, bool capture);

}  // namespace

int set_graphs(int enable) { return g_graphs.exchange(enable ? 1 : 0); }

BatchRunPtr prove_batch_begin(ProveCtx& ctx, int g, const ProveJob* jobs_in, size_t nj, hipStream_t st,
                              bool pipelined) {
  ZK_REQUIRE(nj >= 1, "empty proof batch");
  ZK_REQUIRE(g >= 0 && g < ProveCtx::GENS, "bad context generation");
  ZK_REQUIRE(current_device() == ctx.device, "proof context of another device");
  for (size_t j = 0; j < nj; j++)
    ZK_REQUIRE(jobs_in[j].pk && jobs_in[j].pk->device == ctx.device, "a proving key lives on another device");
  ProveGen& G = ctx.gen[g];
  std::vector<uint64_t> key;
  key.reserve(nj + 2);
  key.push_back((uint64_t)(uintptr_t)st);
  key.push_back(tuning_fingerprint());
  key.push_back(profiling_enabled() ? 1 : 0);
  key.push_back(pipelined ? 1 : 0);
  for (size_t j = 0; j < nj; j++) {
    key.push_back(jobs_in[j].pk->id);
    // device buffers are baked into a captured graph
    key.push_back(jobs_in[j].device_io ? (uint64_t)(uintptr_t)jobs_in[j].X : 0);
    key.push_back(jobs_in[j].device_io ? (uint64_t)(uintptr_t)jobs_in[j].W : 0);
    key.push_back(jobs_in[j].device_io ? (uint64_t)(uintptr_t)jobs_in[j].Y : 0);
  }
  const bool graphs = ctx.graphs && g_graphs.load();
  // graphs run on the context's own stream, after everything queued on the
  // calling stream (which may be the null stream, which cannot be captured)
  hipStream_t gs = ctx.graph_stream;
  auto fork = [&] {
    ZK_HIP(hipEventRecord(G.fork_ev, st));
    ZK_HIP(hipStreamWaitEvent(gs, G.fork_ev, 0));
  };
  auto join = [&] {
    ZK_HIP(hipEventRecord(G.graph_ev, gs));
    ZK_HIP(hipStreamWaitEvent(st, G.graph_ev, 0));
  };
  if (graphs && G.graph && G.graph_key == key) {
    // replay: the same buffers, tables and launches; only X and W change
    BatchRunPtr run(new BatchRun(*G.graph_run));
    BatchRun& R = *run;
    R.jobs.assign(jobs_in, jobs_in + nj);
    R.host_t0 = std::chrono::steady_clock::now();
    R.graphed = true;
    for (size_t j = 0; j < nj; j++) {
      if (jobs_in[j].device_io) continue;  // the buffers are part of the key
      const Layout& L = jobs_in[j].pk->L;
      std::memcpy(R.slots[j].xh, jobs_in[j].X, (size_t)L.a * L.n);
      std::memcpy(R.slots[j].wh, jobs_in[j].W, (size_t)L.n * L.b);
    }
    *R.flag_host = 0u;
    fork();
    ZK_HIP(hipGraphLaunch(G.graph, gs));
    join();
    return run;
  }
  // a new composition rewrites the generation's tables: the graph is stale
  const bool capture = graphs && G.seen_key == key;
  if (G.graph) {
    ZK_HIP(hipGraphExecDestroy(G.graph));
    G.graph = nullptr;
    G.graph_key.clear();
    G.graph_run.reset();
    release_graph_slots(G.graph_prof);
  }
  G.seen_key = key;
  BatchRunPtr run(new BatchRun());
  BatchRun& R = *run;
  R.ctx = &ctx;
  R.g = g;
  R.h_on_main = !pipelined;
  R.jobs.assign(jobs_in, jobs_in + nj);
  R.host_t0 = std::chrono::steady_clock::now();
  while (G.slot_ws.size() < nj) G.slot_ws.emplace_back(new Workspace());
  if (!capture) {
    enqueue_batch(ctx, G, R, st, false);
    return run;
  }
  // the composition ran just before on this generation, so every buffer
  // already has its size: the capture allocates nothing.  The lanes join the
  // capture, so it uses the context's own lane streams (another context's
  // eager work on the shared lanes must not end up in this graph).
  for (int lane = 0; lane < ProveCtx::LANES; lane++)
    if (!ctx.cap_lanes[lane]) ZK_HIP(hipStreamCreateWithFlags(&ctx.cap_lanes[lane], hipStreamNonBlocking));
  fork();
  ZK_HIP(hipStreamBeginCapture(gs, hipStreamCaptureModeRelaxed));
  hipGraph_t graph = nullptr;
  std::vector<int> prof;
  set_capture_sink(&prof);
  try {
    enqueue_batch(ctx, G, R, gs, true);
    for (int lane = 0; lane < ProveCtx::LANES; lane++) {
      ZK_HIP(hipEventRecord(G.join_ev[lane], ctx.cap_lanes[lane]));
      ZK_HIP(hipStreamWaitEvent(gs, G.join_ev[lane], 0));
    }
  } catch (...) {
    set_capture_sink(nullptr);
    release_graph_slots(prof);
    if (hipStreamEndCapture(gs, &graph) == hipSuccess && graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    throw;
  }
  set_capture_sink(nullptr);
  const hipError_t ec = hipStreamEndCapture(gs, &graph);
  if (ec != hipSuccess) release_graph_slots(prof);
  ZK_HIP(ec);
  hipGraphExec_t exec = nullptr;
  const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) release_graph_slots(prof);
  ZK_HIP(e);
  G.graph = exec;
  G.graph_key = key;
  G.graph_prof = std::move(prof);
  R.graphed = true;
  G.graph_run.reset(new BatchRun(R));
  G.graph_run->jobs.clear();
  ZK_HIP(hipGraphLaunch(exec, gs));
  join();
  return run;
}

namespace {

void enqueue_batch(ProveCtx& ctx, ProveGen& G, BatchRun& R, hipStream_t st, bool capture) {
  const ProveJob* jobs = R.jobs.data();
  const size_t nj = R.jobs.size();
  record_ext(G.ev[0], st, capture);

  // ---- witnesses and evaluation vectors (eager: the stage events are bound
  // to the dispatch of the kernels they follow, no marker packets between)
  YCopy ycopy;
  R.slots = enqueue_witness_batch(jobs, nj, G, st, &ycopy, &R.flag_host, !capture, G.ev[1]);
  std::vector<Slot>& slots = R.slots;
  if (capture) record_ext(G.ev[1], st, capture);
  // Each event record on the stream holds its next kernel back by a few
  // microseconds, so eager lanes wait on the stage-timing event itself; under
  // capture the timing events are graph nodes and a plain record carries the
  // dependency.
  if (capture) ZK_HIP(hipEventRecord(G.witness_ev, st));
  const hipEvent_t wit_ev = capture ? G.witness_ev : G.ev[1];
  // ---- MSM jobs of every proof, by lane.  Those that need only the
  // assignment run from the end of the witness on, overlapping the quotient:
  // one pipeline for all G1 queries A, B1, L and one for B2 in G2; the H MSMs
  // follow the quotient on the third lane.
  std::vector<MsmInput> &in_g1 = R.in_g1, &in_g2 = R.in_g2, &in_h = R.in_h;
  std::vector<int> &own_g1 = R.own_g1, &query_g1 = R.query_g1, &own_g2 = R.own_g2, &own_h = R.own_h;
  auto build_lists = [&] {
    for (size_t j = 0; j < nj; j++) {
      for (const MsmJob& m : msm_jobs(jobs[j].pk, slots[j].assign, slots[j].aev, slots[j].wk)) {
        if (m.query == ZKVC_Q_H) {
          in_h.push_back(m.in);
          own_h.push_back((int)j);
        } else if (m.group == 2) {
          in_g2.push_back(m.in);
          own_g2.push_back((int)j);
        } else {
          in_g1.push_back(m.in);
          own_g1.push_back((int)j);
          query_g1.push_back(m.query);
        }
      }
    }
    R.pend_g1.resize(in_g1.size());
    R.pend_g2.resize(in_g2.size());
    R.pend_h.resize(in_h.size());
  };
  const hipStream_t* lanes = capture ? ctx.cap_lanes : ctx.lanes;
  hipStream_t lane_h = lanes[ProveCtx::LANE_H], lane_g1 = lanes[ProveCtx::LANE_G1], lane_g2 = lanes[ProveCtx::LANE_G2];
  auto g2_lane = [&] {
    ZK_HIP(hipStreamWaitEvent(lane_g2, G.wrow_ev, 0));
    msm_enqueue_batch_g2(in_g2.data(), (int)in_g2.size(), G.lane_ws[ProveCtx::LANE_G2], lane_g2, R.pend_g2.data());
    record_ext(G.done_ev[ProveCtx::LANE_G2], lane_g2, capture);
    record_ext(G.lane_t[ProveCtx::LANE_G2], lane_g2, capture);
  };
  auto g1_lane = [&] {
    ZK_HIP(hipStreamWaitEvent(lane_g1, wit_ev, 0));
    msm_enqueue_batch_g1(in_g1.data(), (int)in_g1.size(), G.lane_ws[ProveCtx::LANE_G1], lane_g1, R.pend_g1.data());
    // Y of host-buffer jobs (final since the witness event) at the end of this lane
    if (ycopy.bytes) ZK_HIP(hipMemcpyAsync(ycopy.dst, ycopy.src, ycopy.bytes, hipMemcpyDeviceToHost, lane_g1));
    record_ext(G.done_ev[ProveCtx::LANE_G1], lane_g1, capture);
    record_ext(G.lane_t[ProveCtx::LANE_G1], lane_g1, capture);
  };
  // Every launch costs host time, so one thread enqueueing the lanes one
  // after the other delays the later ones: a helper builds the job lists and
  // enqueues the G2 lane, another the G1 lane once the lists exist, while
  // this thread goes straight on to the quotient and then the H lane (the
  // critical path).  Under capture everything is enqueued from here.
  std::future<void> f_g2, f_g1;
  std::promise<void> lists_ready;
  std::shared_future<void> lists = lists_ready.get_future().share();
  if (capture) {
    build_lists();
    g2_lane();
  } else {
    f_g2 = ctx.pool->run([&] {
      try {
        build_lists();
      } catch (...) {
        lists_ready.set_exception(std::current_exception());
        throw;
      }
      lists_ready.set_value();
      g2_lane();
    });
    f_g1 = ctx.pool->run([&] {
      lists.get();
      g1_lane();
    });
  }
  auto join_helpers = [&] {
    if (f_g2.valid()) f_g2.wait();
    if (f_g1.valid()) f_g1.wait();
  };
  try {
    // ---- QAP quotients: iNTT (DIF, natural -> bit-reversed coefficients),
    // coset NTT (DIT, bit-reversed -> natural evaluations on g H), pointwise
    // (A B - C)/(g^N - 1): h on the coset, the H query's scalars.  Proofs of
    // one domain size share every launch.
    std::map<int, std::vector<size_t>> by_size;
    for (size_t j = 0; j < nj; j++) by_size[jobs[j].pk->L.log_n].push_back(j);
    // device tables for groups of several proofs: (A, B, C) triples
    std::vector<uint32_t*> tab_v;
    std::vector<size_t> tab_off;
    for (auto& kv : by_size) {
      tab_off.push_back(tab_v.size());
      if (kv.second.size() < 2) continue;
      for (size_t j : kv.second) {
        tab_v.push_back(slots[j].aev);
        tab_v.push_back(slots[j].bev);
        tab_v.push_back(slots[j].cev);
      }
    }
    uint32_t** tab_dev = nullptr;
    if (!tab_v.empty()) {
      const size_t bytes = tab_v.size() * sizeof(uint32_t*);
      uint32_t** tab_host = G.shared.host<uint32_t*>(C_TABLE, bytes);
      tab_dev = G.shared.get<uint32_t*>(C_TABLE, bytes);
      std::memcpy(tab_host, tab_v.data(), bytes);
      ZK_HIP(hipMemcpyAsync(tab_dev, tab_host, bytes, hipMemcpyHostToDevice, st));
    }
    size_t gi = 0;
    for (auto& kv : by_size) {
      const int Lg = kv.first;
      const size_t k = kv.second.size();
      const hipEvent_t end_bound = !capture && gi + 1 == by_size.size() ? G.ev[2] : nullptr;
      if (k == 1) {
        const Slot& S = slots[kv.second[0]];
        uint32_t* const vecs[3] = {S.aev, S.bev, S.cev};
        qap_quotient_launch(vecs, nullptr, 1, Lg, st, end_bound);
      } else {
        qap_quotient_launch(nullptr, tab_dev + tab_off[gi], (int)k, Lg, st, end_bound);
      }
      gi++;
    }
    if (capture) record_ext(G.ev[2], st, capture);
    if (capture) ZK_HIP(hipEventRecord(G.quotient_ev, st));

    // ---- the H lane after the quotients
    if (!capture) lists.get();  // rethrows a failure to build the lists
    const hipStream_t h_st = R.h_on_main ? st : lane_h;
    if (!R.h_on_main) ZK_HIP(hipStreamWaitEvent(lane_h, capture ? G.quotient_ev : G.ev[2], 0));
    msm_enqueue_batch_g1(in_h.data(), (int)in_h.size(), G.lane_ws[ProveCtx::LANE_H], h_st, R.pend_h.data(),
                         H_LANE_PRIO);
    record_ext(G.done_ev[ProveCtx::LANE_H], h_st, capture);
    record_ext(G.lane_t[ProveCtx::LANE_H], h_st, capture);
  } catch (...) {
    join_helpers();
    throw;
  }
  if (capture) {
    g1_lane();
  } else {
    join_helpers();  // both finished before either error is rethrown
    f_g2.get();
    f_g1.get();
  }
}

}  // namespace


void prove_batch_finish(ProveCtx& ctx, BatchRun& R) {
  ZK_REQUIRE(!R.finished && R.ctx == &ctx, "batch already finished or of another context");
  R.finished = true;
  ProveGen& G = ctx.gen[R.g];
  const ProveJob* jobs = R.jobs.data();
  const size_t nj = R.jobs.size();
  const std::vector<Slot>& slots = R.slots;
  const std::vector<int> &own_g1 = R.own_g1, &query_g1 = R.query_g1, &own_g2 = R.own_g2, &own_h = R.own_h;
  const std::vector<MsmPending> &pend_g1 = R.pend_g1, &pend_g2 = R.pend_g2, &pend_h = R.pend_h;
  // ---- host side, per lane as each lane completes: the plane sums by
  // Horner's rule, then everything that lane's results allow.  The G1 lane
  // yields A, B1 and s A + r B1 - r s delta (by the G1 endomorphism: half-length
  // scalars, one shared doubling chain per proof of a batch, four threads for a
  // single proof); the G2 lane yields B; the H lane only its sums.
  const size_t nthr = host_threads();
  struct G1Part {
    host::G1J A, L, sA_rB1;
  };
  std::vector<G1Part> g1p(nj);
  std::vector<host::G2J> Bp(nj);
  std::vector<host::G1J> Hp(nj, host::G1J::inf());
  // each proof's MSM results, indexed by lane entry
  std::vector<std::vector<size_t>> g1_of(nj), g2_of(nj);
  for (size_t q = 0; q < own_g1.size(); q++) g1_of[own_g1[q]].push_back(q);
  for (size_t q = 0; q < own_g2.size(); q++) g2_of[own_g2[q]].push_back(q);
  // What needs only r and s (the fixed-base multiples of delta) is done while
  // the lanes run; a single proof also splits s A + r B1 over two threads.
  struct Fixed {
    host::G1J rd1, sd1, rsd1;
    host::G2J sd2;
  };
  std::vector<Fixed> fx(nj);
  auto f_g1 = ctx.pool->run([&] {
    parallel_for(nj, nthr, [&](size_t j) {
      uint64_t rw[4], sw[4], rsw[4];
      jobs[j].r.to_u64(rw);
      jobs[j].s.to_u64(sw);
      host::HFr::mul(jobs[j].r, jobs[j].s).to_u64(rsw);
      fx[j].rd1 = jobs[j].pk->delta1_table.mul(rw);
      fx[j].sd1 = jobs[j].pk->delta1_table.mul(sw);
      fx[j].rsd1 = jobs[j].pk->delta1_table.mul(rsw);
    });
    ZK_HIP(hipEventSynchronize(G.done_ev[ProveCtx::LANE_G1]));
    parallel_for(nj, nthr, [&](size_t j) {
      const ProveJob& J = jobs[j];
      const zkvc_pk* pk = J.pk;
      uint64_t rw[4], sw[4];
      J.r.to_u64(rw);
      J.s.to_u64(sw);
      host::G1J msmA = host::G1J::inf(), msmB1 = host::G1J::inf(), msmL = host::G1J::inf();
      for (size_t q : g1_of[j]) {
        const host::G1J v = msm_finish_g1(pend_g1[q]);
        switch (query_g1[q]) {
          case ZKVC_Q_A: msmA = host::G1J::add(msmA, v); break;
          case ZKVC_Q_B1: msmB1 = host::G1J::add(msmB1, v); break;
          default: msmL = host::G1J::add(msmL, v); break;
        }
      }
      G1Part& o = g1p[j];
      o.A = host::G1J::add(host::G1J::add(pk->alpha1, msmA), fx[j].rd1);
      const host::G1J B1 = host::G1J::add(host::G1J::add(pk->beta1, msmB1), fx[j].sd1);
      host::G1J sArB1;
      if (nj == 1) {  // the four GLV halves of s A and r B1 on four threads
        const host::GlvSplit ss = host::glv_split(sw), rs = host::glv_split(rw);
        host::G1J part[4];
        parallel_for(4, 4, [&](size_t h) {
          part[h] = h < 2 ? host::glv_half(o.A, ss, (int)h) : host::glv_half(B1, rs, (int)h - 2);
        });
        sArB1 = host::G1J::add(host::G1J::add(part[0], part[1]), host::G1J::add(part[2], part[3]));
      } else {
        sArB1 = host::glv_mul2(o.A, sw, B1, rw);
      }
      o.sA_rB1 = host::G1J::add(sArB1, host::G1J::neg(fx[j].rsd1));
      o.L = msmL;
      g1_to_abi(o.A, &J.out->A);  // A is final here (its inversion stays off the H lane's tail)
    });
  });
  auto f_g2 = ctx.pool->run([&] {
    parallel_for(nj, nthr / 2 + 1, [&](size_t j) {
      uint64_t sw[4];
      jobs[j].s.to_u64(sw);
      fx[j].sd2 = jobs[j].pk->delta2_table.mul(sw);
    });
    ZK_HIP(hipEventSynchronize(G.done_ev[ProveCtx::LANE_G2]));
    parallel_for(nj, nthr / 2 + 1, [&](size_t j) {
      host::G2J msmB2 = host::G2J::inf();
      for (size_t q : g2_of[j]) msmB2 = host::G2J::add(msmB2, msm_finish_g2(pend_g2[q]));
      Bp[j] = host::G2J::add(host::G2J::add(jobs[j].pk->beta2, msmB2), fx[j].sd2);
      g2_to_abi(Bp[j], &jobs[j].out->B);
    });
  });
  // the pool's futures do not wait when destroyed: wait for the lane tasks
  // (they use this frame) before leaving it, also when an error unwinds it
  struct WaitAll {
    std::future<void>* f[2];
    ~WaitAll() {
      for (auto* x : f)
        if (x->valid()) x->wait();
    }
  } wait_all{{&f_g1, &f_g2}};
  ZK_HIP(hipEventSynchronize(G.ev[2]));  // witnesses (the row flag) and quotients
  if (*R.flag_host) throw Error(ZKVC_EDEVICE, "internal error: a witness does not satisfy its circuit");
  // The H lane ends the proof: this thread polls for it (no sleeping thread
  // to wake at the end of the device work) and combines its planes.
  for (;;) {
    const hipError_t e = hipEventQuery(G.done_ev[ProveCtx::LANE_H]);
    if (e == hipSuccess) break;
    if (e != hipErrorNotReady) ZK_HIP(e);
  }
  const auto asm_t0 = std::chrono::steady_clock::now();
  parallel_for(own_h.size(), nthr / 2 + 1, [&](size_t q) { Hp[own_h[q]] = msm_finish_g1(pend_h[q]); });
  f_g1.get();
  f_g2.get();
  for (size_t j = 0; j < nj; j++) {
    const Layout& L = jobs[j].pk->L;
    // C = sum_aux a_i L_i + h(tau) t(tau)/delta + s A + r B1 - r s delta
    const host::G1J C = host::G1J::add(host::G1J::add(g1p[j].L, Hp[j]), g1p[j].sA_rB1);
    g1_to_abi(C, &jobs[j].out->C);  // A and B were written by their lanes' tasks
    if (!jobs[j].device_io) std::memcpy(jobs[j].Y, slots[j].yh, (size_t)L.a * L.b * 4);
  }
  const auto host_t1 = std::chrono::steady_clock::now();
  auto ms = [&](hipEvent_t a, hipEvent_t b) {
    float t = 0.f;
    (void)hipEventElapsedTime(&t, a, b);
    return t;
  };
  ctx.last.witness_ms = ms(G.ev[0], G.ev[1]);
  ctx.last.ntt_ms = ms(G.ev[1], G.ev[2]);
  float msm = 0.f;
  for (int lane = 0; lane < ProveCtx::LANES; lane++) msm = std::max(msm, ms(G.ev[2], G.lane_t[lane]));
  ctx.last.msm_ms = msm;
  ctx.last.host_ms = std::chrono::duration<float, std::milli>(host_t1 - asm_t0).count();
  ctx.last.total_ms = std::chrono::duration<float, std::milli>(host_t1 - R.host_t0).count();
  if (R.graphed) collect_graph_slots(G.graph_prof);
}

void prove_batch_abandon(BatchRunPtr& run) {
  if (!run) return;
  if (!run->finished) {
    ProveGen& G = run->ctx->gen[run->g];
    (void)hipEventSynchronize(G.ev[2]);
    for (int lane = 0; lane < ProveCtx::LANES; lane++) (void)hipEventSynchronize(G.done_ev[lane]);
  }
  run.reset();
}

void groth16_prove_batch(ProveCtx& ctx, const ProveJob* jobs, size_t nj, hipStream_t st) {
  BatchRunPtr run = prove_batch_begin(ctx, 0, jobs, nj, st, false);
  try {
    prove_batch_finish(ctx, *run);
  } catch (...) {
    prove_batch_abandon(run);
    throw;
  }
  // the context is idle: buffers replaced while this batch grew its
  // workspaces can go (the graph, if one was captured, uses the current ones)
  run.reset();
  ctx.release_retired();
}



void groth16_prove(zkvc_pk* pk, const int8_t* X, const int8_t* W, const host::HFr& r, const host::HFr& s, int32_t* Y,
                   zkvc_proof* out, hipStream_t st, bool device_io) {
  if (!pk->ctx) pk->ctx.reset(new ProveCtx());
  ProveJob j;
  j.pk = pk;
  j.X = X;
  j.W = W;
  j.r = r;
  j.s = s;
  j.Y = Y;
  j.out = out;
  j.device_io = device_io;
  groth16_prove_batch(*pk->ctx, &j, 1, st);
  pk->last = pk->ctx->last;
}

}  // namespace zkvc

zkvc_pk::~zkvc_pk() = default;
