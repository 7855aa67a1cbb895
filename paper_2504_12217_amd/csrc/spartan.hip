// Spartan (the zkVC-S backend, Section II and Table II) for the CRPC
// circuits: the prover on the GPU, the verifier on the host.
//
// The argument (Spartan's NIZK without zero-knowledge blinding; the paper
// names the backend but fixes neither commitment nor curve):
//   1. the witness half w of z = (witness | constant, x, y), padded to 2^sw,
//      is committed row by row: C_i = sum_col w[i cols + col] G_col;
//   2. sum-check of sum_x eq(tau, x) (Az(x) Bz(x) - Cz(x)) = 0 over the m
//      constraint rows (degree 3, values at 0..3 per round);
//   3. vA, vB, vC = Az~, Bz~, Cz~ at r_x, then rA, rB, rC;
//   4. sum-check of sum_y M(y) z(y) = rA vA + rB vB + rC vC with
//      M(y) = sum_x eq(r_x, x) (rA A + rB B + rC C)[x][y] (degree 2);
//   5. t[col] = sum_row eq(r_row, row) w[row, col], opening w~ at r_y
//      without its top coordinate (square-root commitment layout).
// Every index's bit k is variable k (least significant first); a round binds
// the least significant variable, f[i] <- f[2i] + r (f[2i+1] - f[2i]).
// Fiat-Shamir: state' = SHA-256(state || label || data); a challenge is the
// 512-bit little-endian integer SHA-256(state || label || 00) ||
// SHA-256(state || label || 01) mod r, then state' = SHA-256(state || label || 02).
// The transcript lives in device memory from the first challenge on, so the
// sum-check rounds run with no host round trip.
#include <algorithm>
#include <array>
#include <cstring>
#include <memory>
#include <mutex>
#include <vector>

#include "api_common.hpp"
#include "curve.hpp"
#include "field.hpp"
#include "msm.hpp"
#include "prover.hpp"
#include "sha256.hpp"

namespace zkvc {
namespace {

constexpr int SC_THREADS = 256;      // multi-block round kernels
constexpr int TAIL_THREADS = 512;    // the last rounds, one block
constexpr uint64_t TAIL_LEN = 2048;  // arrays of at most this length finish in the tail kernel
constexpr int MAX_SC_BLOCKS = 1024;

// ------------------------------------------------------------------ sizes
struct SpSizes {
  Layout L;
  uint64_t m = 0, ell = 0, nv = 0, nw = 0, half = 0, cols = 0, rows = 0;
  int sx = 0, sw = 0, sy = 0, col_bits = 0, row_bits = 0;
  size_t proof_bytes() const { return rows * 64 + (size_t)sx * 4 * 32 + 96 + (size_t)sy * 3 * 32 + cols * 32; }
};

int log2_ceil(uint64_t v) {
  int k = 0;
  while ((1ull << k) < v) k++;
  return k;
}

SpSizes sp_sizes(uint32_t a, uint32_t n, uint32_t b, uint32_t kind) {
  ZK_REQUIRE(kind == ZKVC_CRPC_PSQ || kind == ZKVC_CRPC, "the Spartan prover supports the CRPC kinds");
  SpSizes S;
  S.L = r1cs_layout(a, n, b, kind);
  S.m = S.L.m;
  S.ell = S.L.ell;
  S.nv = S.L.nv;
  S.nw = S.nv - S.ell - 1;
  S.sx = std::max(1, log2_ceil(S.m));
  S.sw = std::max({1, log2_ceil(S.nw), log2_ceil(S.ell + 1)});
  S.sy = S.sw + 1;
  ZK_REQUIRE(S.sy <= 30, "Spartan instance too large");
  S.half = 1ull << S.sw;
  S.col_bits = (S.sw + 1) / 2;
  S.row_bits = S.sw - S.col_bits;
  S.cols = 1ull << S.col_bits;
  S.rows = 1ull << S.row_bits;
  return S;
}

// ------------------------------------------------------------------ device transcript
__device__ void fr_to_bytes(const Fr& x_mont, uint8_t out[32]) {
  uint32_t w[8];
  Fr::from_mont(x_mont).pack(w);
#pragma unroll
  for (int k = 0; k < 8; k++) {
    out[4 * k] = (uint8_t)w[k];
    out[4 * k + 1] = (uint8_t)(w[k] >> 8);
    out[4 * k + 2] = (uint8_t)(w[k] >> 16);
    out[4 * k + 3] = (uint8_t)(w[k] >> 24);
  }
}

__device__ Fr fr_from_bytes_wide(const uint8_t b[32]) {  // any 256-bit value, reduced, Montgomery form
  uint32_t w[8];
#pragma unroll
  for (int k = 0; k < 8; k++)
    w[k] = (uint32_t)b[4 * k] | ((uint32_t)b[4 * k + 1] << 8) | ((uint32_t)b[4 * k + 2] << 16) |
           ((uint32_t)b[4 * k + 3] << 24);
  return Fr::to_mont(Fr::unpack(w));
}

// the challenge of the current state under `label`, advancing the state
__device__ Fr tr_challenge(uint8_t st[32], const char* label) {
  uint8_t lo[32], hi[32];
  uint8_t tag = 0;
  sha256_chain_copy(st, label, &tag, 1, lo);
  tag = 1;
  sha256_chain_copy(st, label, &tag, 1, hi);
  tag = 2;
  sha256_chain(st, label, &tag, 1);
  // 2^256 mod r in Montgomery form: (2^128)^2
  uint32_t w128[8] = {0, 0, 0, 0, 1, 0, 0, 0};
  const Fr t128 = Fr::to_mont(Fr::unpack(w128));
  const Fr k256 = Fr::mul(t128, t128);
  return Fr::add(fr_from_bytes_wide(lo), Fr::mul(fr_from_bytes_wide(hi), k256));
}

// ------------------------------------------------------------------ small kernels
// tau_0 .. tau_{count-1} from the transcript (one thread)
__global__ void k_sp_challenges(uint8_t* state, int count, uint32_t* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  uint8_t st[32];
  for (int k = 0; k < 32; k++) st[k] = state[k];
  for (int k = 0; k < count; k++) tr_challenge(st, "tau").store(out + 8 * k);
  for (int k = 0; k < 32; k++) state[k] = st[k];
}

// out[i] = eq(r, bits(i)) = prod_k (r_k if bit k of i else 1 - r_k), i < 2^s
__global__ void k_sp_eq_table(const uint32_t* r, int s, uint64_t n, uint32_t* out) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  Fr acc = Fr::one();
  for (int k = 0; k < s; k++) {
    const Fr rk = Fr::load(r + 8 * k);
    acc = Fr::mul(acc, ((i >> k) & 1) ? rk : Fr::sub(Fr::one(), rk));
  }
  acc.store(out + 8 * i);
}

// z in Montgomery form: the witness variables, zero padding, then the
// constant and the public x and y at 2^sw
__global__ void k_sp_zvec(const uint32_t* assign, uint64_t ell, uint64_t nw, uint64_t half, uint32_t* Z) {
  const uint64_t y = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (y >= 2 * half) return;
  Fr v = Fr::zero();
  if (y < half) {
    if (y < nw) v = Fr::to_mont(Fr::load(assign + 8 * (ell + 1 + y)));
  } else if (y - half <= ell) {
    v = Fr::to_mont(Fr::load(assign + 8 * (y - half)));
  }
  v.store(Z + 8 * y);
}

// Az, Bz, Cz rows (canonical, m of them) into Montgomery arrays of length len
__global__ void k_sp_abc(const uint32_t* aev, const uint32_t* bev, const uint32_t* cev, uint64_t m, uint64_t len,
                         uint32_t* A, uint32_t* B, uint32_t* C) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  const bool in = i < m;
  (in ? Fr::to_mont(Fr::load(aev + 8 * i)) : Fr::zero()).store(A + 8 * i);
  (in ? Fr::to_mont(Fr::load(bev + 8 * i)) : Fr::zero()).store(B + 8 * i);
  (in ? Fr::to_mont(Fr::load(cev + 8 * i)) : Fr::zero()).store(C + 8 * i);
}

// M(y) for the CRPC kinds (rows k < n: A = z^(ib) x_ik, B = z^j w_kj;
// CRPC_PSQ: C_k = s_k - s_(k-1), C_(n-1) = Y(z) - s_(n-2);
// CRPC: C_k = P_k, last row (sum_k P_k) * 1 = Y(z)).
struct MParams {
  uint32_t kind, a, n, b;
  uint64_t ell, half, len;
  const uint32_t* ex;     // eq(r_x, x), 2^sx entries
  const uint32_t* rabc;   // rA, rB, rC
  const uint32_t* zpow;   // z^e, e < a b
};
__global__ void k_sp_m(MParams p, uint32_t* M) {
  const uint64_t y = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (y >= p.len) return;
  const Fr rA = Fr::load(p.rabc), rB = Fr::load(p.rabc + 8), rC = Fr::load(p.rabc + 16);
  auto ex = [&](uint64_t x) { return Fr::load(p.ex + 8 * x); };
  auto zp = [&](uint64_t e) { return Fr::load(p.zpow + 8 * e); };
  const uint64_t nb = (uint64_t)p.n * p.b, an = (uint64_t)p.a * p.n, n = p.n, b = p.b;
  Fr v = Fr::zero();
  if (y < p.half) {
    if (y < nb) {  // w_kj
      const uint64_t k = y / b, j = y % b;
      v = Fr::mul(Fr::mul(rB, ex(k)), zp(j));
    } else if (p.kind == ZKVC_CRPC_PSQ && y - nb + 1 < n) {  // s_t, t < n - 1
      const uint64_t t = y - nb;
      v = Fr::mul(rC, Fr::sub(ex(t), ex(t + 1)));
    } else if (p.kind == ZKVC_CRPC && y - nb < n) {  // P_t
      const uint64_t t = y - nb;
      v = Fr::add(Fr::mul(rC, ex(t)), Fr::mul(rA, ex(n)));
    }
  } else {
    const uint64_t t = y - p.half;
    if (t == 0) {
      if (p.kind == ZKVC_CRPC) v = Fr::mul(rB, ex(n));
    } else if (t <= an) {  // x_ik
      const uint64_t i = (t - 1) / n, k = (t - 1) % n;
      v = Fr::mul(Fr::mul(rA, ex(k)), zp(i * b));
    } else if (t <= p.ell) {  // y_ij, in the last row
      const uint64_t e = t - 1 - an;
      v = Fr::mul(Fr::mul(rC, ex(p.kind == ZKVC_CRPC ? n : n - 1)), zp(e));
    }
  }
  v.store(M + 8 * y);
}

// t[col] = sum_row er[row] w[row cols + col]: partial sums over chunks of rows
__global__ void k_sp_hyrax(const uint32_t* Z, const uint32_t* er, uint64_t rows, uint64_t cols, uint32_t chunk,
                           uint32_t* part) {
  const uint64_t col = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= cols) return;
  const uint64_t r0 = (uint64_t)blockIdx.y * chunk, r1 = std::min<uint64_t>(rows, r0 + chunk);
  Fr acc = Fr::zero();
  for (uint64_t r = r0; r < r1; r++) acc = Fr::add(acc, Fr::mul(Fr::load(er + 8 * r), Fr::load(Z + 8 * (r * cols + col))));
  acc.store(part + 8 * (blockIdx.y * cols + col));
}
__global__ void k_sp_hyrax_sum(const uint32_t* part, uint32_t nchunk, uint64_t cols, uint32_t* t_out) {
  const uint64_t col = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= cols) return;
  Fr acc = Fr::zero();
  for (uint32_t c = 0; c < nchunk; c++) acc = Fr::add(acc, Fr::load(part + 8 * (c * cols + col)));
  Fr::from_mont(acc).store(t_out + 8 * col);
}

// ------------------------------------------------------------------ sum-check
// DEG 3: arrays E, A, B, C and terms e (a b - c); DEG 2: arrays M, Z and terms m z.
template <int DEG>
struct Sc {
  static constexpr int NA = DEG == 3 ? 4 : 2;
  const uint32_t* in[4];
  uint32_t* out[4];
};

template <int DEG>
__device__ __forceinline__ void sc_accumulate(const Fr* lo, const Fr* hi, Fr* g) {
  constexpr int NA = Sc<DEG>::NA;
  Fr cur[NA], d[NA];
#pragma unroll
  for (int q = 0; q < NA; q++) {
    cur[q] = lo[q];
    d[q] = Fr::sub(hi[q], lo[q]);
  }
#pragma unroll
  for (int t = 0; t <= DEG; t++) {
    if (DEG == 3)
      g[t] = Fr::add(g[t], Fr::mul(cur[0], Fr::sub(Fr::mul(cur[1], cur[2]), cur[3])));
    else
      g[t] = Fr::add(g[t], Fr::mul(cur[0], cur[1]));
    if (t < DEG) {
#pragma unroll
      for (int q = 0; q < NA; q++) cur[q] = Fr::add(cur[q], d[q]);
    }
  }
}

template <int NT>
__device__ Fr block_reduce(Fr x, uint32_t* sh) {
  for (int o = NT / 2; o >= 1; o >>= 1) {
    if ((int)threadIdx.x >= o && (int)threadIdx.x < 2 * o) {
#pragma unroll
      for (int q = 0; q < NL; q++) sh[(threadIdx.x - o) * NL + q] = x.v[q];
    }
    __syncthreads();
    if ((int)threadIdx.x < o) {
      Fr y;
#pragma unroll
      for (int q = 0; q < NL; q++) y.v[q] = sh[threadIdx.x * NL + q];
      x = Fr::add(x, y);
    }
    __syncthreads();
  }
  return x;
}

// per-block sums of the round polynomial's values over pairs i < half
template <int DEG>
__global__ void __launch_bounds__(SC_THREADS) k_sc_partial(Sc<DEG> A, uint64_t half, uint32_t* part) {
  constexpr int NA = Sc<DEG>::NA;
  __shared__ uint32_t sh[SC_THREADS / 2 * NL];
  Fr g[DEG + 1];
#pragma unroll
  for (int t = 0; t <= DEG; t++) g[t] = Fr::zero();
  for (uint64_t i = (uint64_t)blockIdx.x * SC_THREADS + threadIdx.x; i < half; i += (uint64_t)gridDim.x * SC_THREADS) {
    Fr lo[NA], hi[NA];
#pragma unroll
    for (int q = 0; q < NA; q++) {
      lo[q] = Fr::load(A.in[q] + 16 * i);
      hi[q] = Fr::load(A.in[q] + 16 * i + 8);
    }
    sc_accumulate<DEG>(lo, hi, g);
  }
#pragma unroll
  for (int t = 0; t <= DEG; t++) {
    g[t] = block_reduce<SC_THREADS>(g[t], sh);
    if (threadIdx.x == 0) g[t].store(part + 8 * ((uint64_t)blockIdx.x * (DEG + 1) + t));
  }
}

// the round's values from the block sums: into the proof (canonical), into
// the transcript; the round challenge into r_out (Montgomery)
template <int DEG>
__global__ void __launch_bounds__(SC_THREADS) k_sc_finish(const uint32_t* part, uint32_t nblocks, uint8_t* state,
                                                          uint32_t* proof_g, uint32_t* r_out) {
  __shared__ uint32_t sh[SC_THREADS / 2 * NL];
  __shared__ uint32_t gsh[(DEG + 1) * NL];
  for (int t = 0; t <= DEG; t++) {
    Fr acc = Fr::zero();
    for (uint32_t bl = threadIdx.x; bl < nblocks; bl += SC_THREADS)
      acc = Fr::add(acc, Fr::load(part + 8 * ((uint64_t)bl * (DEG + 1) + t)));
    acc = block_reduce<SC_THREADS>(acc, sh);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int q = 0; q < NL; q++) gsh[t * NL + q] = acc.v[q];
    }
  }
  if (threadIdx.x != 0) return;
  uint8_t st[32], msg[(DEG + 1) * 32];
  for (int k = 0; k < 32; k++) st[k] = state[k];
  for (int t = 0; t <= DEG; t++) {
    Fr g;
#pragma unroll
    for (int q = 0; q < NL; q++) g.v[q] = gsh[t * NL + q];
    Fr::from_mont(g).store(proof_g + 8 * t);
    fr_to_bytes(g, msg + 32 * t);
  }
  sha256_chain(st, DEG == 3 ? "sc1" : "sc2", msg, sizeof(msg));
  tr_challenge(st, DEG == 3 ? "r1" : "r2").store(r_out);
  for (int k = 0; k < 32; k++) state[k] = st[k];
}

template <int DEG>
__global__ void k_sc_fold(Sc<DEG> A, uint64_t half, const uint32_t* r_in) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= half) return;
  const Fr r = Fr::load(r_in);
#pragma unroll
  for (int q = 0; q < Sc<DEG>::NA; q++) {
    const Fr lo = Fr::load(A.in[q] + 16 * i), hi = Fr::load(A.in[q] + 16 * i + 8);
    Fr::add(lo, Fr::mul(r, Fr::sub(hi, lo))).store(A.out[q] + 8 * i);
  }
}

// The remaining rounds in one block (len <= TAIL_LEN), ping-ponging between
// in and out.  After the last round of sum-check 1 the block also records
// vA, vB, vC and draws rA, rB, rC (into r_after).
template <int DEG>
__global__ void __launch_bounds__(TAIL_THREADS) k_sc_tail(Sc<DEG> A, uint64_t len, uint8_t* state, uint32_t* proof_g,
                                                          uint32_t* r_out, uint32_t* proof_after, uint32_t* r_after) {
  constexpr int NA = Sc<DEG>::NA;
  __shared__ uint32_t sh[TAIL_THREADS / 2 * NL];
  __shared__ uint32_t gsh[(DEG + 1) * NL];
  __shared__ uint32_t rsh[NL];
  const uint32_t* src[NA];
  uint32_t* dst[NA];
#pragma unroll
  for (int q = 0; q < NA; q++) {
    src[q] = A.in[q];
    dst[q] = A.out[q];
  }
  int round = 0;
  for (uint64_t n = len; n > 1; n >>= 1, round++) {
    const uint64_t half = n >> 1;
    Fr g[DEG + 1];
#pragma unroll
    for (int t = 0; t <= DEG; t++) g[t] = Fr::zero();
    for (uint64_t i = threadIdx.x; i < half; i += TAIL_THREADS) {
      Fr lo[NA], hi[NA];
#pragma unroll
      for (int q = 0; q < NA; q++) {
        lo[q] = Fr::load(src[q] + 16 * i);
        hi[q] = Fr::load(src[q] + 16 * i + 8);
      }
      sc_accumulate<DEG>(lo, hi, g);
    }
#pragma unroll
    for (int t = 0; t <= DEG; t++) {
      g[t] = block_reduce<TAIL_THREADS>(g[t], sh);
      if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NL; q++) gsh[t * NL + q] = g[t].v[q];
      }
    }
    if (threadIdx.x == 0) {
      uint8_t st[32], msg[(DEG + 1) * 32];
      for (int k = 0; k < 32; k++) st[k] = state[k];
      for (int t = 0; t <= DEG; t++) {
        Fr gt;
#pragma unroll
        for (int q = 0; q < NL; q++) gt.v[q] = gsh[t * NL + q];
        Fr::from_mont(gt).store(proof_g + 8 * ((uint64_t)round * (DEG + 1) + t));
        fr_to_bytes(gt, msg + 32 * t);
      }
      sha256_chain(st, DEG == 3 ? "sc1" : "sc2", msg, sizeof(msg));
      const Fr r = tr_challenge(st, DEG == 3 ? "r1" : "r2");
      r.store(r_out + 8 * round);
#pragma unroll
      for (int q = 0; q < NL; q++) rsh[q] = r.v[q];
      for (int k = 0; k < 32; k++) state[k] = st[k];
    }
    __syncthreads();
    Fr r;
#pragma unroll
    for (int q = 0; q < NL; q++) r.v[q] = rsh[q];
    for (uint64_t i = threadIdx.x; i < half; i += TAIL_THREADS) {
#pragma unroll
      for (int q = 0; q < NA; q++) {
        const Fr lo = Fr::load(src[q] + 16 * i), hi = Fr::load(src[q] + 16 * i + 8);
        Fr::add(lo, Fr::mul(r, Fr::sub(hi, lo))).store(dst[q] + 8 * i);
      }
    }
    __threadfence_block();
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NA; q++) {
      const uint32_t* t = src[q];
      src[q] = dst[q];
      dst[q] = const_cast<uint32_t*>(t);
    }
  }
  if (DEG != 3 || threadIdx.x != 0 || proof_after == nullptr) return;
  // vA, vB, vC: the folded A, B, C
  uint8_t st[32], msg[96];
  for (int k = 0; k < 32; k++) st[k] = state[k];
  for (int q = 0; q < 3; q++) {
    const Fr v = Fr::load(src[1 + q]);
    Fr::from_mont(v).store(proof_after + 8 * q);
    fr_to_bytes(v, msg + 32 * q);
  }
  sha256_chain(st, "vabc", msg, 96);
  tr_challenge(st, "ra").store(r_after);
  tr_challenge(st, "rb").store(r_after + 8);
  tr_challenge(st, "rc").store(r_after + 16);
  for (int k = 0; k < 32; k++) state[k] = st[k];
}

}  // namespace
}  // namespace zkvc

// ------------------------------------------------------------------ host side
struct zkvc_spartan_key {
  int device = 0;
  zkvc::SpSizes S;
  zkvc::host::HFr z;
  zkvc::DevBuf gens;  // cols affine points, device layout
  zkvc::DevBuf zpow;  // z^e, e < a b, device layout
  std::vector<zkvc_g1> gens_host;
  zkvc::Workspace ws;
  std::mutex mu;
};

namespace zkvc {
namespace {

enum SpSlot {
  SP_X = 200, SP_W, SP_Y, SP_ASSIGN, SP_AEV, SP_BEV, SP_CEV, SP_Z, SP_ARR0, SP_ARR1, SP_ARR2, SP_ARR3, SP_ARR4,
  SP_ARR5, SP_ARR6, SP_ARR7, SP_M, SP_ZS, SP_M2, SP_Z2, SP_PART, SP_STATE, SP_R, SP_PROOF, SP_EX, SP_ER, SP_HY
};

void put_fr_bytes(const host::HFr& v, uint8_t out[32]) {
  uint32_t w[8];
  v.to_u32(w);
  std::memcpy(out, w, 32);  // little-endian host
}

struct HostTranscript {
  uint8_t st[32];
  HostTranscript() {
    const char* d = "zkvc-spartan-v1";
    Sha256 s;
    s.init();
    s.update(reinterpret_cast<const uint8_t*>(d), std::strlen(d));
    s.final(st);
  }
  void absorb(const char* label, const uint8_t* data, size_t n) { sha256_chain(st, label, data, n); }
  host::HFr challenge(const char* label) {
    uint8_t lo[32], hi[32], tag = 0;
    sha256_chain_copy(st, label, &tag, 1, lo);
    tag = 1;
    sha256_chain_copy(st, label, &tag, 1, hi);
    tag = 2;
    sha256_chain(st, label, &tag, 1);
    uint64_t a[4], b[4];
    std::memcpy(a, lo, 32);
    std::memcpy(b, hi, 32);
    const uint64_t w128[4] = {0, 0, 1, 0};
    const host::HFr t128 = host::HFr::from_u64(w128);
    return host::HFr::add(host::HFr::from_u64(a), host::HFr::mul(host::HFr::from_u64(b), host::HFr::sqr(t128)));
  }
};

std::vector<uint8_t> io_bytes(const SpSizes& S, const int8_t* X, const int32_t* Y) {
  const size_t an = (size_t)S.L.a * S.L.n, ab = (size_t)S.L.a * S.L.b;
  std::vector<uint8_t> out(an + 4 * ab);
  std::memcpy(out.data(), X, an);
  std::memcpy(out.data() + an, Y, 4 * ab);  // little-endian host
  return out;
}

HostTranscript start_transcript(const SpSizes& S, const host::HFr& z, const int8_t* X, const int32_t* Y,
                                const uint8_t* comm_bytes) {
  HostTranscript tr;
  uint8_t head[48];
  const uint32_t dims[4] = {S.L.a, S.L.n, S.L.b, S.L.kind};
  std::memcpy(head, dims, 16);
  put_fr_bytes(z, head + 16);
  tr.absorb("shape", head, 48);
  const std::vector<uint8_t> io = io_bytes(S, X, Y);
  tr.absorb("io", io.data(), io.size());
  tr.absorb("comm", comm_bytes, S.rows * 64);
  return tr;
}

void enqueue_eq(const uint32_t* r, int s, uint32_t* out, hipStream_t st) {
  const uint64_t n = 1ull << s;
  hipLaunchKernelGGL(k_sp_eq_table, dim3(cdiv(n, 256)), dim3(256), 0, st, r, s, n, out);
  ZK_HIP(hipGetLastError());
}

// One sum-check over arrays of length len = 2^rounds (in[q]), with scratch
// buffers b1[q], b2[q] of length len / 2; proof_g receives (DEG + 1) values
// per round, r_out one challenge per round.
template <int DEG>
void run_sumcheck(const uint32_t* const* in, uint32_t* const* b1, uint32_t* const* b2, uint64_t len, uint8_t* state,
                  uint32_t* part, uint32_t* proof_g, uint32_t* r_out, uint32_t* proof_after, uint32_t* r_after,
                  hipStream_t st) {
  constexpr int NA = Sc<DEG>::NA;
  Sc<DEG> A{};
  for (int q = 0; q < NA; q++) {
    A.in[q] = in[q];
    A.out[q] = b1[q];
  }
  int round = 0;
  bool use_b1 = true;
  while (len > TAIL_LEN) {
    const uint64_t half = len / 2;
    const unsigned blocks = (unsigned)std::min<uint64_t>(MAX_SC_BLOCKS, cdiv(half, SC_THREADS));
    hipLaunchKernelGGL(k_sc_partial<DEG>, dim3(blocks), dim3(SC_THREADS), 0, st, A, half, part);
    ZK_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sc_finish<DEG>, dim3(1), dim3(SC_THREADS), 0, st, part, blocks, state,
                       proof_g + 8 * (DEG + 1) * round, r_out + 8 * round);
    ZK_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sc_fold<DEG>, dim3(cdiv(half, 256)), dim3(256), 0, st, A, half, r_out + 8 * round);
    ZK_HIP(hipGetLastError());
    for (int q = 0; q < NA; q++) {
      A.in[q] = A.out[q];
      A.out[q] = use_b1 ? b2[q] : b1[q];
    }
    use_b1 = !use_b1;
    len = half;
    round++;
  }
  hipLaunchKernelGGL(k_sc_tail<DEG>, dim3(1), dim3(TAIL_THREADS), 0, st, A, len, state,
                     proof_g + 8 * (DEG + 1) * round, r_out + 8 * round, proof_after, r_after);
  ZK_HIP(hipGetLastError());
}

// Jacobian points to canonical affine encodings with one field inversion
void batch_affine_host(const std::vector<host::G1J>& pts, uint8_t* out) {
  const size_t n = pts.size();
  std::vector<host::HFq> pre(n);
  host::HFq acc = host::HFq::one();
  for (size_t i = 0; i < n; i++) {
    pre[i] = acc;
    if (!pts[i].is_inf()) acc = host::HFq::mul(acc, pts[i].Z);
  }
  host::HFq inv = host::HFq::inv(acc);
  for (size_t i = n; i-- > 0;) {
    uint8_t* o = out + 64 * i;
    if (pts[i].is_inf()) {
      std::memset(o, 0, 64);
      continue;
    }
    const host::HFq zi = host::HFq::mul(inv, pre[i]);
    inv = host::HFq::mul(inv, pts[i].Z);
    const host::HFq zi2 = host::HFq::sqr(zi);
    const host::HFq x = host::HFq::mul(pts[i].X, zi2), y = host::HFq::mul(pts[i].Y, host::HFq::mul(zi2, zi));
    uint32_t w[8];
    x.to_u32(w);
    std::memcpy(o, w, 32);
    y.to_u32(w);
    std::memcpy(o + 32, w, 32);
  }
}

void spartan_prove(zkvc_spartan_key* K, const int8_t* X, const int8_t* W, int32_t* Y_out, uint8_t* proof,
                   hipStream_t st) {
  const SpSizes& S = K->S;
  const Layout& L = S.L;
  Workspace& ws = K->ws;
  const size_t an = (size_t)L.a * L.n, nb = (size_t)L.n * L.b, ab = (size_t)L.a * L.b;
  const uint64_t lenx = 1ull << S.sx, leny = 1ull << S.sy;
  // every buffer first
  int8_t* xh = ws.host<int8_t>(SP_X, an + nb);
  int8_t* xd = ws.get<int8_t>(SP_X, an + nb);
  int32_t* yh = ws.host<int32_t>(SP_Y, ab * 4);
  int32_t* yd = ws.get<int32_t>(SP_Y, ab * 4);
  uint32_t* assign = ws.get(SP_ASSIGN, L.nv * 32);
  uint32_t* aev = ws.get(SP_AEV, L.m * 32);
  uint32_t* bev = ws.get(SP_BEV, L.m * 32);
  uint32_t* cev = ws.get(SP_CEV, L.m * 32);
  uint32_t* Z = ws.get(SP_Z, leny * 32);
  uint32_t* arr[8];
  for (int q = 0; q < 8; q++) arr[q] = ws.get(SP_ARR0 + q, (q < 4 ? lenx : lenx / 2 + 1) * 32);
  uint32_t* M = ws.get(SP_M, leny * 32);
  uint32_t* Zs = ws.get(SP_ZS, leny * 32);  // the copy of z that sum-check 2 consumes
  uint32_t* M2 = ws.get(SP_M2, (leny / 2) * 32);
  uint32_t* Z2 = ws.get(SP_Z2, (leny / 2) * 32);
  uint32_t* part = ws.get(SP_PART, (size_t)MAX_SC_BLOCKS * 4 * 32);
  uint8_t* state_h = ws.host<uint8_t>(SP_STATE, 32);
  uint8_t* state_d = ws.get<uint8_t>(SP_STATE, 32);
  // device scalars: tau (sx), r_x (sx), rA rB rC, r_y (sy)
  uint32_t* rv = ws.get(SP_R, (size_t)(2 * S.sx + 3 + S.sy) * 32);
  uint32_t *tau = rv, *rx = rv + 8 * S.sx, *rabc = rv + 16 * S.sx, *ry = rabc + 24;
  // proof values after the commitments (canonical words)
  const size_t nvals = (size_t)S.sx * 4 + 3 + (size_t)S.sy * 3 + S.cols;
  uint32_t* pv_d = ws.get(SP_PROOF, nvals * 32);
  uint32_t* pv_h = ws.host<uint32_t>(SP_PROOF, nvals * 32);
  uint32_t *sc1 = pv_d, *vabc = sc1 + 8 * 4 * S.sx, *sc2 = vabc + 24, *tv = sc2 + 8 * 3 * S.sy;
  uint32_t* ex = ws.get(SP_EX, lenx * 32);
  uint32_t* er = ws.get(SP_ER, S.rows * 32);
  const uint32_t hy_chunks = (uint32_t)std::min<uint64_t>(S.rows, 32);
  uint32_t* hy = ws.get(SP_HY, (size_t)hy_chunks * S.cols * 32);
  // the row commitments' MSM inputs
  std::vector<MsmInput> jobs(S.rows);
  for (uint64_t i = 0; i < S.rows; i++) {
    MsmInput& in = jobs[i];
    const uint64_t lo = i * S.cols;
    in.points = K->gens.get();
    in.npoints = S.cols;
    in.scalars = Z + 8 * lo;
    in.nscalars = lo < S.nw ? S.cols : 0;  // rows past the witness are zero
    in.scalars_mont = true;
    in.max_bits = lo + S.cols <= nb ? 7 : 253;  // |w| <= 2^7; the auxiliary values are full width
  }
  std::vector<MsmPending> pend(S.rows);

  // ---- witness
  std::memcpy(xh, X, an);
  std::memcpy(xh + an, W, nb);
  ZK_HIP(hipMemcpyAsync(xd, xh, an + nb, hipMemcpyHostToDevice, st));
  enqueue_witness_one(L, K->zpow.get(), L.m, xd, xd + an, yd, assign, aev, bev, cev, ws, st);
  ZK_HIP(hipMemcpyAsync(yh, yd, ab * 4, hipMemcpyDeviceToHost, st));
  hipLaunchKernelGGL(k_sp_zvec, dim3(cdiv(leny, 256)), dim3(256), 0, st, assign, S.ell, S.nw, S.half, Z);
  ZK_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_sp_abc, dim3(cdiv(lenx, 256)), dim3(256), 0, st, aev, bev, cev, (uint64_t)L.m, lenx, arr[1],
                     arr[2], arr[3]);
  ZK_HIP(hipGetLastError());
  // ---- row commitments
  msm_enqueue_batch_g1(jobs.data(), (int)S.rows, ws, st, pend.data());
  ZK_HIP(hipStreamSynchronize(st));
  std::memcpy(Y_out, yh, ab * 4);
  std::vector<host::G1J> comm(S.rows);
  for (uint64_t i = 0; i < S.rows; i++) comm[i] = msm_finish_g1(pend[i]);
  batch_affine_host(comm, proof);
  HostTranscript tr = start_transcript(S, K->z, X, Y_out, proof);
  std::memcpy(state_h, tr.st, 32);
  ZK_HIP(hipMemcpyAsync(state_d, state_h, 32, hipMemcpyHostToDevice, st));
  // ---- sum-check 1
  hipLaunchKernelGGL(k_sp_challenges, dim3(1), dim3(64), 0, st, state_d, S.sx, tau);
  ZK_HIP(hipGetLastError());
  enqueue_eq(tau, S.sx, arr[0], st);
  {
    const uint32_t* in[4] = {arr[0], arr[1], arr[2], arr[3]};
    uint32_t* b1[4] = {arr[4], arr[5], arr[6], arr[7]};
    uint32_t* b2[4] = {arr[0], arr[1], arr[2], arr[3]};  // the input arrays are free after the first fold
    // with len > TAIL_LEN the multi-block rounds alternate b1 and b2 (b2 is
    // first written in the second round, after the first fold read in)
    run_sumcheck<3>(in, b1, b2, lenx, state_d, part, sc1, rx, vabc, rabc, st);
  }
  // ---- sum-check 2
  enqueue_eq(rx, S.sx, ex, st);
  {
    MParams mp{L.kind, L.a, L.n, L.b, S.ell, S.half, leny, ex, rabc, K->zpow.get()};
    hipLaunchKernelGGL(k_sp_m, dim3(cdiv(leny, 256)), dim3(256), 0, st, mp, M);
    ZK_HIP(hipGetLastError());
    // z is still needed by the opening: sum-check 2 runs on a copy (the
    // rounds fold into their inputs' buffers once those are consumed)
    ZK_HIP(hipMemcpyAsync(Zs, Z, leny * 32, hipMemcpyDeviceToDevice, st));
    const uint32_t* in[2] = {M, Zs};
    uint32_t* b1[2] = {M2, Z2};
    uint32_t* b2[2] = {M, Zs};
    run_sumcheck<2>(in, b1, b2, leny, state_d, part, sc2, ry, nullptr, nullptr, st);
  }
  // ---- opening: t[col] = sum_row eq(r_row, row) w[row, col]
  enqueue_eq(ry + 8 * S.col_bits, S.row_bits, er, st);
  {
    const uint32_t chunk = (uint32_t)cdiv(S.rows, hy_chunks);
    hipLaunchKernelGGL(k_sp_hyrax, dim3(cdiv(S.cols, 256), hy_chunks), dim3(256), 0, st, Z, er, S.rows, S.cols, chunk,
                       hy);
    ZK_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sp_hyrax_sum, dim3(cdiv(S.cols, 256)), dim3(256), 0, st, hy, hy_chunks, S.cols, tv);
    ZK_HIP(hipGetLastError());
  }
  ZK_HIP(hipMemcpyAsync(pv_h, pv_d, nvals * 32, hipMemcpyDeviceToHost, st));
  ZK_HIP(hipStreamSynchronize(st));
  std::memcpy(proof + S.rows * 64, pv_h, nvals * 32);  // canonical little-endian words
}

}  // namespace
}  // namespace zkvc

namespace zkvc {
namespace {

bool fr_from_bytes_checked(const uint8_t* p, host::HFr& out) {
  uint32_t w[8];
  std::memcpy(w, p, 32);
  if (!host::HFr::canonical_ok(w)) return false;
  out = host::HFr::from_u32(w);
  return true;
}

// the point encoded at p (canonical affine, all-zero = infinity); false if off the curve or not canonical
bool g1_from_bytes_checked(const uint8_t* p, host::G1J& out) {
  uint32_t x[8], y[8];
  std::memcpy(x, p, 32);
  std::memcpy(y, p + 32, 32);
  bool zero = true;
  for (int k = 0; k < 8; k++) zero = zero && x[k] == 0 && y[k] == 0;
  if (zero) {
    out = host::G1J::inf();
    return true;
  }
  if (!host::HFq::canonical_ok(x) || !host::HFq::canonical_ok(y)) return false;
  const host::HFq X = host::HFq::from_u32(x), Y = host::HFq::from_u32(y);
  const host::HFq rhs = host::HFq::add(host::HFq::mul(host::HFq::sqr(X), X), host::HFq::from_uint(3));
  if (host::HFq::sqr(Y) != rhs) return false;
  out = host::G1J::from_affine(X, Y);
  return true;
}

// sum_i s_i P_i by 8-bit windows and running bucket sums (host)
host::G1J host_msm(const std::vector<host::G1J>& pts, const std::vector<host::HFr>& sc) {
  const size_t n = pts.size();
  std::vector<std::array<uint8_t, 32>> digits(n);
  for (size_t i = 0; i < n; i++) {
    uint64_t w[4];
    sc[i].to_u64(w);
    std::memcpy(digits[i].data(), w, 32);
  }
  host::G1J acc = host::G1J::inf();
  std::vector<host::G1J> bucket(255);
  for (int win = 31; win >= 0; win--) {
    for (int k = 0; k < 8; k++) acc = host::G1J::dbl(acc);
    for (auto& b : bucket) b = host::G1J::inf();
    for (size_t i = 0; i < n; i++) {
      const uint8_t d = digits[i][win];
      if (d && !pts[i].is_inf()) bucket[d - 1] = host::G1J::add(bucket[d - 1], pts[i]);
    }
    host::G1J run = host::G1J::inf(), tot = host::G1J::inf();
    for (int d = 254; d >= 0; d--) {
      run = host::G1J::add(run, bucket[d]);
      tot = host::G1J::add(tot, run);
    }
    acc = host::G1J::add(acc, tot);
  }
  return acc;
}

// [eq(r, i) for i < 2^len(r)]
std::vector<host::HFr> eq_table_host(const host::HFr* r, int s) {
  std::vector<host::HFr> t(1, host::HFr::one());
  for (int k = 0; k < s; k++) {
    const host::HFr one_minus = host::HFr::sub(host::HFr::one(), r[k]);
    std::vector<host::HFr> u(t.size() * 2);
    for (size_t i = 0; i < t.size(); i++) {
      u[i] = host::HFr::mul(t[i], one_minus);              // bit k = 0
      u[i + t.size()] = host::HFr::mul(t[i], r[k]);         // bit k = 1
    }
    t.swap(u);
  }
  return t;
}

// eq(r, y) for every y < 2^s from two half tables
struct EqSplit {
  int h = 0;
  std::vector<host::HFr> lo, hi;
  EqSplit(const std::vector<host::HFr>& r) {
    const int s = (int)r.size();
    h = s / 2;
    lo = eq_table_host(r.data(), h);
    hi = eq_table_host(r.data() + h, s - h);
  }
  host::HFr at(uint64_t y) const { return host::HFr::mul(lo[y & ((1ull << h) - 1)], hi[y >> h]); }
};

host::HFr interp(const host::HFr* g, int npts, const host::HFr& r) {
  using host::HFr;
  const HFr one = HFr::one(), two = HFr::from_uint(2), three = HFr::from_uint(3);
  const HFr r1 = HFr::sub(r, one), r2 = HFr::sub(r, two), r3 = HFr::sub(r, three);
  if (npts == 3) {  // nodes 0, 1, 2
    const HFr inv2 = HFr::inv(two);
    const HFr L0 = HFr::mul(HFr::mul(r1, r2), inv2);
    const HFr L1 = HFr::neg(HFr::mul(r, r2));
    const HFr L2 = HFr::mul(HFr::mul(r, r1), inv2);
    return HFr::add(HFr::add(HFr::mul(g[0], L0), HFr::mul(g[1], L1)), HFr::mul(g[2], L2));
  }
  const HFr inv2 = HFr::inv(two), inv6 = HFr::inv(HFr::from_uint(6));  // nodes 0, 1, 2, 3
  const HFr L0 = HFr::neg(HFr::mul(HFr::mul(HFr::mul(r1, r2), r3), inv6));
  const HFr L1 = HFr::mul(HFr::mul(HFr::mul(r, r2), r3), inv2);
  const HFr L2 = HFr::neg(HFr::mul(HFr::mul(HFr::mul(r, r1), r3), inv2));
  const HFr L3 = HFr::mul(HFr::mul(HFr::mul(r, r1), r2), inv6);
  return HFr::add(HFr::add(HFr::mul(g[0], L0), HFr::mul(g[1], L1)), HFr::add(HFr::mul(g[2], L2), HFr::mul(g[3], L3)));
}

host::HFr fr_int(int64_t v) {
  const host::HFr a = host::HFr::from_uint((uint64_t)(v < 0 ? -v : v));
  return v < 0 ? host::HFr::neg(a) : a;
}

int spartan_verify(const SpSizes& S, const host::HFr& z, const zkvc_g1* gens, const int8_t* X, const int32_t* Y,
                   const uint8_t* proof) {
  using host::HFr;
  const Layout& L = S.L;
  const uint64_t an = (uint64_t)L.a * L.n, ab = (uint64_t)L.a * L.b, nb = (uint64_t)L.n * L.b, n = L.n, b = L.b;
  // parse
  std::vector<host::G1J> comm(S.rows), gen(S.cols);
  for (uint64_t i = 0; i < S.rows; i++)
    if (!g1_from_bytes_checked(proof + 64 * i, comm[i])) return 0;
  for (uint64_t i = 0; i < S.cols; i++)
    if (!g1_from_bytes_checked(reinterpret_cast<const uint8_t*>(&gens[i]), gen[i])) return 0;
  const uint8_t* vals = proof + S.rows * 64;
  const size_t nvals = (size_t)S.sx * 4 + 3 + (size_t)S.sy * 3 + S.cols;
  std::vector<HFr> v(nvals);
  for (size_t i = 0; i < nvals; i++)
    if (!fr_from_bytes_checked(vals + 32 * i, v[i])) return 0;
  const HFr* sc1 = v.data();
  const HFr* vabc = sc1 + 4 * S.sx;
  const HFr* sc2 = vabc + 3;
  const HFr* t = sc2 + 3 * S.sy;
  // sum-check 1
  HostTranscript tr = start_transcript(S, z, X, Y, proof);
  std::vector<HFr> tau(S.sx), rx(S.sx), ry(S.sy);
  for (int k = 0; k < S.sx; k++) tau[k] = tr.challenge("tau");
  HFr claim = HFr::zero();
  for (int j = 0; j < S.sx; j++) {
    const HFr* g = sc1 + 4 * j;
    if (HFr::add(g[0], g[1]) != claim) return 0;
    tr.absorb("sc1", vals + 32 * 4 * j, 128);
    rx[j] = tr.challenge("r1");
    claim = interp(g, 4, rx[j]);
  }
  HFr eqt = HFr::one();
  for (int k = 0; k < S.sx; k++)
    eqt = HFr::mul(eqt, HFr::add(HFr::mul(tau[k], rx[k]),
                                 HFr::mul(HFr::sub(HFr::one(), tau[k]), HFr::sub(HFr::one(), rx[k]))));
  if (claim != HFr::mul(eqt, HFr::sub(HFr::mul(vabc[0], vabc[1]), vabc[2]))) return 0;
  tr.absorb("vabc", vals + 32 * 4 * S.sx, 96);
  const HFr ra = tr.challenge("ra"), rb = tr.challenge("rb"), rc = tr.challenge("rc");
  claim = HFr::add(HFr::add(HFr::mul(ra, vabc[0]), HFr::mul(rb, vabc[1])), HFr::mul(rc, vabc[2]));
  // sum-check 2
  for (int j = 0; j < S.sy; j++) {
    const HFr* g = sc2 + 3 * j;
    if (HFr::add(g[0], g[1]) != claim) return 0;
    tr.absorb("sc2", vals + 32 * (4 * S.sx + 3 + 3 * j), 96);
    ry[j] = tr.challenge("r2");
    claim = interp(g, 3, ry[j]);
  }
  // z~(r_y): the opened witness part and the public part
  const std::vector<HFr> rp(ry.begin(), ry.begin() + S.sw);
  const HFr rtop = ry[S.sw];
  const std::vector<HFr> ec = eq_table_host(rp.data(), S.col_bits);
  HFr vw = HFr::zero();
  for (uint64_t c = 0; c < S.cols; c++) vw = HFr::add(vw, HFr::mul(t[c], ec[c]));
  const EqSplit eqp(rp);
  HFr pe = eqp.at(0);  // the constant 1
  for (uint64_t i = 0; i < an; i++) pe = HFr::add(pe, HFr::mul(fr_int(X[i]), eqp.at(1 + i)));
  for (uint64_t i = 0; i < ab; i++) pe = HFr::add(pe, HFr::mul(fr_int(Y[i]), eqp.at(1 + an + i)));
  const HFr ze = HFr::add(HFr::mul(HFr::sub(HFr::one(), rtop), vw), HFr::mul(rtop, pe));
  // M~(r_y) from the CRPC rows' closed form
  const std::vector<HFr> ex = eq_table_host(rx.data(), S.sx);
  const EqSplit eqy(ry);
  std::vector<HFr> zp(ab);
  {
    HFr acc = HFr::one();
    for (uint64_t e = 0; e < ab; e++) {
      zp[e] = acc;
      acc = HFr::mul(acc, z);
    }
  }
  const bool psq = L.kind == ZKVC_CRPC_PSQ;
  const uint64_t last = psq ? n - 1 : n;
  HFr mt = HFr::zero();
  for (uint64_t k = 0; k < n; k++) {  // w_kj
    const HFr rk = HFr::mul(rb, ex[k]);
    HFr s = HFr::zero();
    for (uint64_t j = 0; j < b; j++) s = HFr::add(s, HFr::mul(zp[j], eqy.at(k * b + j)));
    mt = HFr::add(mt, HFr::mul(rk, s));
  }
  for (uint64_t tt = 0; tt < (psq ? n - 1 : n); tt++) {  // auxiliary
    const HFr m = psq ? HFr::mul(rc, HFr::sub(ex[tt], ex[tt + 1])) : HFr::add(HFr::mul(rc, ex[tt]), HFr::mul(ra, ex[n]));
    mt = HFr::add(mt, HFr::mul(m, eqy.at(nb + tt)));
  }
  if (!psq) mt = HFr::add(mt, HFr::mul(HFr::mul(rb, ex[n]), eqy.at(S.half)));  // the constant
  for (uint64_t i = 0; i < L.a; i++) {  // x_ik
    const HFr ri = HFr::mul(ra, zp[i * b]);
    for (uint64_t k = 0; k < n; k++) mt = HFr::add(mt, HFr::mul(HFr::mul(ri, ex[k]), eqy.at(S.half + 1 + i * n + k)));
  }
  {
    const HFr rl = HFr::mul(rc, ex[last]);
    for (uint64_t e = 0; e < ab; e++) mt = HFr::add(mt, HFr::mul(HFr::mul(rl, zp[e]), eqy.at(S.half + 1 + an + e)));
  }
  if (claim != HFr::mul(mt, ze)) return 0;
  // the opening against the row commitments: sum t_c G_c - sum eq(r_row, i) C_i = 0
  const std::vector<HFr> er = eq_table_host(rp.data() + S.col_bits, S.row_bits);
  std::vector<host::G1J> pts(gen);
  std::vector<HFr> sc(t, t + S.cols);
  for (uint64_t i = 0; i < S.rows; i++) {
    pts.push_back(comm[i]);
    sc.push_back(HFr::neg(er[i]));
  }
  return host_msm(pts, sc).is_inf() ? 1 : 0;
}

}  // namespace
}  // namespace zkvc

using namespace zkvc;

extern "C" {

int zkvc_spartan_info(const zkvc_shape* shape, zkvc_spartan_info_t* out) {
  return guarded([&] {
    ZK_REQUIRE(shape && out, "null argument");
    const SpSizes S = sp_sizes(shape->a, shape->n, shape->b, shape->kind);
    out->constraints = S.m;
    out->sx = (uint32_t)S.sx;
    out->sy = (uint32_t)S.sy;
    out->rows = (uint32_t)S.rows;
    out->cols = (uint32_t)S.cols;
    out->proof_bytes = S.proof_bytes();
  });
}

int zkvc_spartan_setup(const zkvc_shape* shape, const zkvc_fr* z, const zkvc_g1* gens, size_t ngens,
                       zkvc_spartan_key** key_out, void* hip_stream) {
  return guarded([&] {
    ZK_REQUIRE(shape && z && gens && key_out, "null argument");
    const SpSizes S = sp_sizes(shape->a, shape->n, shape->b, shape->kind);
    ZK_REQUIRE(ngens == S.cols, "the commitment needs exactly zkvc_spartan_info().cols generators");
    const host::HFr zz = fr_in(*z, "z");
    ZK_REQUIRE(!zz.is_zero(), "z must be nonzero");
    for (size_t i = 0; i < ngens; i++) {
      host::G1J p;
      ZK_REQUIRE(g1_from_bytes_checked(reinterpret_cast<const uint8_t*>(&gens[i]), p) && !p.is_inf(),
                 "generators must be points of G1 other than infinity");
    }
    hipStream_t st = (hipStream_t)hip_stream;
    std::unique_ptr<zkvc_spartan_key> K(new zkvc_spartan_key());
    K->device = current_device();
    K->S = S;
    K->z = zz;
    K->gens_host.assign(gens, gens + ngens);
    // generators in the device layout
    K->gens.alloc(ngens * 64);
    {
      DevBuf tmp(ngens * 64);
      ZK_HIP(hipMemcpyAsync(tmp.get(), gens, ngens * 64, hipMemcpyHostToDevice, st));
      points_to_mont_g1(tmp.get(), K->gens.get(), ngens, st);
      ZK_HIP(hipStreamSynchronize(st));
    }
    const uint32_t cnt = S.L.a * S.L.b;
    K->zpow.alloc((size_t)cnt * 32);
    {
      uint32_t zw[8];
      zz.to_dev(zw);
      DevBuf dz(32);
      ZK_HIP(hipMemcpyAsync(dz.get(), zw, 32, hipMemcpyHostToDevice, st));
      enqueue_zpow(dz.get(), cnt, K->zpow.get(), st);
      ZK_HIP(hipStreamSynchronize(st));
    }
    *key_out = K.release();
  });
}

int zkvc_spartan_key_free(zkvc_spartan_key* key) {
  return guarded([&] { delete key; });
}

int zkvc_spartan_prove(zkvc_spartan_key* key, const int8_t* X, const int8_t* W, int32_t* Y_out, uint8_t* proof,
                       size_t proof_len, void* hip_stream) {
  return guarded([&] {
    ZK_REQUIRE(key && X && W && Y_out && proof, "null argument");
    ZK_REQUIRE(proof_len == key->S.proof_bytes(), "proof buffer must hold exactly zkvc_spartan_info().proof_bytes");
    ZK_REQUIRE(current_device() == key->device, "the Spartan key lives on another device");
    std::lock_guard<std::mutex> lock(key->mu);
    spartan_prove(key, X, W, Y_out, proof, (hipStream_t)hip_stream);
  });
}

int zkvc_spartan_verify(const zkvc_shape* shape, const zkvc_fr* z, const zkvc_g1* gens, size_t ngens,
                        const int8_t* X, const int32_t* Y, const uint8_t* proof, size_t proof_len) {
  int result = 0;
  const int rc = guarded([&] {
    ZK_REQUIRE(shape && z && gens && X && Y && proof, "null argument");
    const SpSizes S = sp_sizes(shape->a, shape->n, shape->b, shape->kind);
    ZK_REQUIRE(ngens == S.cols, "the commitment needs exactly zkvc_spartan_info().cols generators");
    if (proof_len != S.proof_bytes()) return;  // not a proof of this shape: reject
    result = spartan_verify(S, fr_in(*z, "z"), gens, X, Y, proof);
  });
  return rc < 0 ? rc : result;
}

}  // extern "C"
