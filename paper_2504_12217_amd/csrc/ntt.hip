// Fr number-theoretic transforms for the QAP quotient (iNTT, coset NTT, pointwise).
//
// A transform of N = 2^L points runs as a sequence of in-place passes (the
// four-step decomposition of Bailey applied recursively).  Pass j owns a
// contiguous bit range of the element address: for every setting of the other
// bits ("group") it performs a 2^k-point radix-2 transform in LDS over that
// bit range, then multiplies by the inter-pass twiddles.  With address
//   a = hi * M + t * 2^B + g     (M = 2^(B+k), t < 2^k, g < 2^B)
// a decimation-in-frequency (DIF) pass leaves position t holding frequency
// bitrev_k(t) of its group and then multiplies it by omega_M^(g * bitrev_k(t)).
// Running DIF passes from the top bit range down yields the full transform in
// bit-reversed order.  The decimation-in-time (DIT) transform is the exact
// transpose: passes from the bottom bit range up, twiddle first, then DIT
// butterflies, mapping bit-reversed input to natural-order output.
//
// Memory: elements are 32 bytes (8 words).  A workgroup stages 1024 elements
// (its groups, chosen so that global loads and stores come in runs of
// consecutive addresses) in LDS as 29-bit limbs, 36 bytes each.
//
// Values inside a transform are lazy: any representative in [0, 2m) of the
// residue (sums and differences fold back below 2m with one conditional
// step, products skip their final subtraction, and a DIF difference that
// meets a twiddle goes into the product as a - b + 2m unreduced).  The last
// pass of a transform stores canonical values.
#include "ntt.hpp"

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "field.hpp"
#include "host_field.hpp"
#include "profile.hpp"
#include "tune.hpp"
#include "util.hpp"

namespace zkvc {

constexpr int NTT_MAX_K = 10;
constexpr int NTT_E = 1 << NTT_MAX_K;  // elements per workgroup
constexpr int NTT_THREADS = NTT_E / 2;
constexpr int POW_BITS = NTT_POW_BITS;
constexpr int MAX_LOG = NTT_MAX_LOG;
constexpr int TOP_MAX_K = 9;  // fused top pass: 3 regions of at most 2^9 elements

struct PassParams {
  uint32_t* data[NTT_MAX_BATCH];  // one vector per blockIdx.y ...
  uint32_t* const* table;         // ... or, if set, a device table of vectors
  int log_n, log_m, k, log_g;
  int dit, inverse, twiddle;
  const uint32_t* tw;             // this pass's twiddles, entry (t << B) | g, or null: power tables
  int first, last;
  int pre_mont, pre_coset, pre_bitrev;
  int post_canon, post_coset, post_bitrev;
  const uint32_t* pre_const;
  const uint32_t* post_const;
  const uint32_t* post_table;     // if set: the last pass's only output factor, entry = address
};

__device__ __forceinline__ void lds_put(uint32_t* lds, uint32_t slot, const Fr& x) {
#pragma unroll
  for (int q = 0; q < NL; q++) lds[slot * NL + q] = x.v[q];
}
__device__ __forceinline__ Fr lds_get(const uint32_t* lds, uint32_t slot) {
  Fr x;
#pragma unroll
  for (int q = 0; q < NL; q++) x.v[q] = lds[slot * NL + q];
  return x;
}

// Stage twiddles are stored as the nine 29-bit limbs the arithmetic uses
// (12 words, 48 bytes: three 16-byte loads), so no unpacking per butterfly.
constexpr uint32_t LOCAL_WORDS = 12;
__device__ __forceinline__ Fr load_limbs(const uint32_t* p) {
  const uint4 a = reinterpret_cast<const uint4*>(p)[0];
  const uint4 b = reinterpret_cast<const uint4*>(p)[1];
  const uint32_t c = p[8];
  return Fr{{a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c}};
}

// The k radix-2 stages of a pass on `nreg` consecutive LDS regions of E
// elements (E / 2^k groups of 2^k each); every thread of the block must call.
__device__ __forceinline__ void lds_stages(uint32_t* lds, int k, uint32_t E, int nreg, bool dit, const uint32_t* local_tab) {
  const uint32_t K = 1u << k;
  const uint32_t half = K >> 1;
  const uint32_t* local = k > 0 ? local_tab + LOCAL_WORDS * (half - 1u) : local_tab;
  const uint32_t nb = (E / 2) * (uint32_t)nreg;
  for (int st = 0; st < k; st++) {
    const int s = dit ? st : (k - 1 - st);
    const uint32_t smask = (1u << s) - 1u;
    for (uint32_t bi = threadIdx.x; bi < nb; bi += blockDim.x) {
      const uint32_t gl = bi >> (k - 1);  // group across all regions (regions are whole groups)
      const uint32_t j = bi & (half - 1u);
      const uint32_t t0 = ((j >> s) << (s + 1)) | (j & smask);
      const uint32_t t1 = t0 | (1u << s);
      const uint32_t widx = (j & smask) << (k - 1 - s);
      // lazy values in [0, 2m) (see the header)
      Fr a = lds_get(lds, gl * K + t0);
      Fr b = lds_get(lds, gl * K + t1);
      if (dit) {
        if (widx) b = Fr::mul_lz(b, load_limbs(local + LOCAL_WORDS * widx));
        const Fr u = Fr::add_lz(a, b);
        const Fr v = Fr::sub_lz(a, b);
        a = u;
        b = v;
      } else {
        const Fr u = Fr::add_lz(a, b);
        const Fr v = widx ? Fr::mul_lz(Fr::sub_nr(a, b), load_limbs(local + LOCAL_WORDS * widx)) : Fr::sub_lz(a, b);
        a = u;
        b = v;
      }
      lds_put(lds, gl * K + t0, a);
      lds_put(lds, gl * K + t1, b);
    }
    __syncthreads();
  }
}

// Element e of a block of pass (k, log_g, B = log_m - k): its group slot gl,
// its position t inside the 2^k-point sub-transform, and its address.
__device__ __forceinline__ uint32_t pass_addr(uint32_t e, int k, int log_g, int B, int log_m, uint32_t gamma0,
                                              uint32_t* gl_out, uint32_t* t_out, uint32_t* g_out) {
  uint32_t gl, t;
  if (B == 0) {
    gl = e >> k;
    t = e & ((1u << k) - 1u);
  } else {
    gl = e & ((1u << log_g) - 1u);
    t = e >> log_g;
  }
  const uint32_t gamma = gamma0 + gl;
  const uint32_t g = gamma & ((1u << B) - 1u);
  *gl_out = gl;
  *t_out = t;
  *g_out = g;
  return ((gamma >> B) << log_m) | (t << B) | g;
}

// The transforms of a proof's quotient lie on its critical path (the H MSM
// waits for them) while the G1 and G2 MSMs run beside them: their waves take
// instruction issue first on a shared SIMD.
constexpr bool NTT_PRIO = true;
__device__ __forceinline__ void ntt_wave_priority() {
  if (NTT_PRIO) __builtin_amdgcn_s_setprio(2);
}

__global__ void __launch_bounds__(NTT_THREADS) k_ntt_pass(PassParams p, NttTables T) {
  extern __shared__ uint32_t lds[];
  ntt_wave_priority();
  const int k = p.k;
  const uint32_t K = 1u << k;
  const uint32_t G = 1u << p.log_g;
  const uint32_t E = K * G;
  const int B = p.log_m - k;
  const uint32_t gmask = (1u << B) - 1u;
  const uint32_t gamma0 = blockIdx.x * G;
  const int tw_shift = MAX_LOG - p.log_m;
  uint32_t* const data = p.table ? p.table[blockIdx.y] : p.data[blockIdx.y];

  // ---- load (global -> registers -> LDS), with first-pass fusions and DIT twiddles
  for (uint32_t e = threadIdx.x; e < E; e += blockDim.x) {
    uint32_t gl, t;
    if (B == 0) {
      gl = e >> k;
      t = e & (K - 1u);
    } else {
      gl = e & (G - 1u);
      t = e >> p.log_g;
    }
    const uint32_t gamma = gamma0 + gl;
    const uint32_t g = gamma & gmask;
    const uint32_t addr = ((gamma >> B) << p.log_m) | (t << B) | g;
    Fr x = Fr::load(data + 8ull * addr);
    if (p.first) {
      if (p.pre_mont) x = Fr::to_mont(x);
      if (p.pre_coset) {
        const uint32_t idx = p.pre_bitrev ? bitrev_bits(addr, p.log_n) : addr;
        x = Fr::mul(x, pow_lookup(T.g[p.pre_coset < 0 ? 1 : 0], idx));
      }
      if (p.pre_const) x = Fr::mul(x, Fr::load(p.pre_const));
    }
    if (p.dit && p.twiddle) {
      const uint32_t ex = g * bitrev_bits(t, k);
      if (ex) x = Fr::mul_lz(x, p.tw ? Fr::load(p.tw + 8u * ((t << B) | g)) : pow_lookup(T.w[p.inverse], ex << tw_shift));
    }
    lds_put(lds, gl * K + t, x);
  }
  __syncthreads();

  // ---- radix-2 stages in LDS
  lds_stages(lds, k, E, 1, p.dit, T.local[p.inverse]);

  // ---- store, with DIF twiddles and last-pass fusions
  for (uint32_t e = threadIdx.x; e < E; e += blockDim.x) {
    uint32_t gl, t;
    if (B == 0) {
      gl = e >> k;
      t = e & (K - 1u);
    } else {
      gl = e & (G - 1u);
      t = e >> p.log_g;
    }
    const uint32_t gamma = gamma0 + gl;
    const uint32_t g = gamma & gmask;
    const uint32_t addr = ((gamma >> B) << p.log_m) | (t << B) | g;
    Fr x = lds_get(lds, gl * K + t);
    if (!p.dit && p.twiddle) {
      const uint32_t ex = g * bitrev_bits(t, k);
      if (ex) x = Fr::mul_lz(x, p.tw ? Fr::load(p.tw + 8u * ((t << B) | g)) : pow_lookup(T.w[p.inverse], ex << tw_shift));
    }
    if (p.last && p.post_table) {
      x = Fr::mul(x, Fr::load(p.post_table + 8ull * addr));
      if (p.post_canon) x = Fr::from_mont(x);
    } else if (p.last) {
      if (p.post_coset) {
        const uint32_t idx = p.post_bitrev ? bitrev_bits(addr, p.log_n) : addr;
        x = Fr::mul(x, pow_lookup(T.g[p.post_coset < 0 ? 1 : 0], idx));
      }
      if (p.post_const) x = Fr::mul(x, Fr::load(p.post_const));
      if (p.post_canon) x = Fr::from_mont(x);
    }
    if (p.last) x = Fr::canon(x);  // a lazy value leaves the transform canonical
    x.store(data + 8ull * addr);
  }
}

// ---- fused passes of the QAP quotient chain.  The inverse transform's last
// pass and the coset transform's first pass cover the same (bottom) bit
// range, so one block does both with the coset scaling between them; the
// coset transform's last pass (the top bit range) and the pointwise quotient
// are done by one block for a proof's A, B and C.  The chain ends there: the
// quotient h stays as its values on the coset, the scalars of an H query
// held in that coset's Lagrange basis.
struct FusedParams {
  uint32_t* data[3];          // one proof's A, B, C ...
  uint32_t* const* table;     // ... or a device table, 3 entries per proof
  int log_n, k, log_g;
  const uint32_t* ninv;       // N^-1 (bottom: with the coset scaling)
  const uint32_t* zinv;       // (g^N - 1)^-1 (top: the pointwise quotient)
  const uint32_t* tw[1];      // top: the pass's forward twiddle table, or null
  const uint32_t* coset;      // bottom: g^bitrev(i) / N by address i, or null
};

// Bottom fusion, one vector per blockIdx.y (A, B, C of each proof in turn).
__global__ void __launch_bounds__(NTT_THREADS) k_ntt_fused_bottom(FusedParams p, NttTables T) {
  extern __shared__ uint32_t lds[];
  ntt_wave_priority();
  const int k = p.k;
  const uint32_t E = 1u << (k + p.log_g);
  const uint32_t gamma0 = blockIdx.x << p.log_g;
  uint32_t* const data = p.table ? p.table[blockIdx.y] : p.data[blockIdx.y];
  uint32_t gl, t, g;
  for (uint32_t e = threadIdx.x; e < E; e += blockDim.x) {
    const uint32_t addr = pass_addr(e, k, p.log_g, 0, k, gamma0, &gl, &t, &g);
    lds_put(lds, gl * (1u << k) + t, Fr::load(data + 8ull * addr));
  }
  __syncthreads();
  lds_stages(lds, k, E, 1, false, T.local[1]);  // inverse DIF, last pass (no twiddle)
  const Fr ninv = Fr::load(p.ninv);
  for (uint32_t e = threadIdx.x; e < E; e += blockDim.x) {
    const uint32_t addr = pass_addr(e, k, p.log_g, 0, k, gamma0, &gl, &t, &g);
    const uint32_t slot = gl * (1u << k) + t;
    // coefficient bitrev(addr) of the inverse transform times g^i / N
    const Fr x = p.coset ? Fr::mul_lz(lds_get(lds, slot), Fr::load(p.coset + 8ull * addr))
                         : Fr::mul_lz(Fr::mul_lz(lds_get(lds, slot), pow_lookup(T.g[0], bitrev_bits(addr, p.log_n))), ninv);
    lds_put(lds, slot, x);
  }
  __syncthreads();
  lds_stages(lds, k, E, 1, true, T.local[0]);  // forward DIT, first pass (no twiddle)
  for (uint32_t e = threadIdx.x; e < E; e += blockDim.x) {
    const uint32_t addr = pass_addr(e, k, p.log_g, 0, k, gamma0, &gl, &t, &g);
    lds_get(lds, gl * (1u << k) + t).store(data + 8ull * addr);
  }
}

// Top fusion, one proof per blockIdx.y: the coset transform's last pass on
// A, B and C, then the pointwise quotient, which overwrites A: h(g omega^a) at
// address a (natural order; lazy values in [0, 2r), device Montgomery form).
__global__ void __launch_bounds__(NTT_THREADS) k_ntt_fused_top(FusedParams p, NttTables T) {
  extern __shared__ uint32_t lds[];
  ntt_wave_priority();
  const int k = p.k, L = p.log_n, B = L - k;
  const uint32_t K = 1u << k;
  const uint32_t E = 1u << (k + p.log_g);
  const uint32_t gamma0 = blockIdx.x << p.log_g;
  const int tw_shift = MAX_LOG - L;
  uint32_t* vec[3];
#pragma unroll
  for (int v = 0; v < 3; v++) vec[v] = p.table ? p.table[3 * blockIdx.y + v] : p.data[v];
  uint32_t gl, t, g;
  const int log_e = k + p.log_g;
  for (uint32_t e = threadIdx.x; e < 3 * E; e += blockDim.x) {
    const uint32_t v = e >> log_e, el = e & (E - 1u);
    const uint32_t addr = pass_addr(el, k, p.log_g, B, L, gamma0, &gl, &t, &g);
    Fr x = Fr::load(vec[v] + 8ull * addr);
    const uint32_t ex = g * bitrev_bits(t, k);  // forward DIT twiddle first
    if (ex) x = Fr::mul_lz(x, p.tw[0] ? Fr::load(p.tw[0] + 8u * ((t << B) | g)) : pow_lookup(T.w[0], ex << tw_shift));
    lds_put(lds, v * E + gl * K + t, x);
  }
  __syncthreads();
  lds_stages(lds, k, E, 3, true, T.local[0]);  // forward DIT, last pass, on A, B and C
  const Fr zinv = Fr::load(p.zinv);
  for (uint32_t e = threadIdx.x; e < E; e += blockDim.x) {
    const uint32_t addr = pass_addr(e, k, p.log_g, B, L, gamma0, &gl, &t, &g);
    const uint32_t slot = gl * K + t;
    const Fr a = lds_get(lds, slot), b = lds_get(lds, E + slot), c = lds_get(lds, 2 * E + slot);
    Fr::mul_lz(Fr::sub_nr(Fr::mul_lz(a, b), c), zinv).store(vec[0] + 8ull * addr);
  }
}

// Twiddles of one pass: entry (t << B) | g = omega_M^(g bitrev_k(t)) (M = 2^(B+k),
// omega of the direction), read in the same order as the pass reads its data.
__global__ void k_twiddle_table(uint32_t* out, int log_m, int k, int dir, NttTables T) {
  const uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >> log_m) return;
  const int B = log_m - k;
  const uint32_t t = idx >> B, g = idx & ((1u << B) - 1u);
  const uint32_t ex = g * bitrev_bits(t, k);
  pow_lookup(T.w[dir], ex << (MAX_LOG - log_m)).store(out + 8ull * idx);
}

// Coset factors of the quotient by address a: g^(+-bitrev(a)) / N, with the
// sign of dir (0: +, 1: -) and N = 2^log_n.
__global__ void k_coset_table(uint32_t* out, int log_n, int dir, NttTables T) {
  const uint32_t a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >> log_n) return;
  Fr::mul(pow_lookup(T.g[dir], bitrev_bits(a, log_n)), Fr::load(T.ninv + 8 * log_n)).store(out + 8ull * a);
}

__global__ void k_bitrev(uint32_t* data, int log_n, uint32_t n) {
  const uint32_t a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  const uint32_t b = bitrev_bits(a, log_n);
  if (a < b) {
    uint4* pa = reinterpret_cast<uint4*>(data + 8ull * a);
    uint4* pb = reinterpret_cast<uint4*>(data + 8ull * b);
    const uint4 a0 = pa[0], a1 = pa[1], b0 = pb[0], b1 = pb[1];
    pa[0] = b0;
    pa[1] = b1;
    pb[0] = a0;
    pb[1] = a1;
  }
}

// ------------------------------------------------------------------ host side
namespace {

struct DeviceTables {
  DevBuf buf;
  NttTables t;
};

void pow_table_host(const host::HFr& base, std::vector<uint32_t>& lo, std::vector<uint32_t>& hi) {
  const int n = 1 << POW_BITS;
  lo.resize(8 * n);
  hi.resize(8 * n);
  host::HFr x = host::HFr::one();
  for (int i = 0; i < n; i++) {
    x.to_dev(&lo[8 * i]);
    x = host::HFr::mul(x, base);
  }
  // x = base^(2^14)
  const host::HFr step = x;
  host::HFr y = host::HFr::one();
  for (int i = 0; i < n; i++) {
    y.to_dev(&hi[8 * i]);
    y = host::HFr::mul(y, step);
  }
}

DeviceTables* build_tables() {
  using host::HFr;
  // omega_{2^28} = 5^((r-1)/2^28)
  uint64_t e[4];
  {
    // (r - 1) >> 28
    uint64_t rm1[4] = {FrParams::P64[0] - 1, FrParams::P64[1], FrParams::P64[2], FrParams::P64[3]};
    for (int k = 0; k < 4; k++) e[k] = (rm1[k] >> 28) | (k < 3 ? (rm1[k + 1] << 36) : 0);
  }
  const HFr five = HFr::from_uint(5);
  const HFr w = HFr::pow(five, e);
  const HFr wi = HFr::inv(w);
  const HFr gi = HFr::inv(five);
  std::vector<uint32_t> tabs[8];
  pow_table_host(w, tabs[0], tabs[1]);
  pow_table_host(wi, tabs[2], tabs[3]);
  pow_table_host(five, tabs[4], tabs[5]);
  pow_table_host(gi, tabs[6], tabs[7]);
  // local tables: omega_{2^k}^j for k = 1..10, j < 2^(k-1), at entry 2^(k-1) - 1 + j,
  // each as nine 29-bit limbs in 12 words
  std::vector<uint32_t> loc[2];
  for (int dir = 0; dir < 2; dir++) {
    loc[dir].assign(LOCAL_WORDS * ((1 << NTT_MAX_K) - 1), 0);
    for (int k = 1; k <= NTT_MAX_K; k++) {
      HFr wk = dir == 0 ? w : wi;
      for (int q = k; q < MAX_LOG; q++) wk = HFr::sqr(wk);  // omega_{2^k}
      HFr x = HFr::one();
      const int off = (1 << (k - 1)) - 1;
      for (int j = 0; j < (1 << (k - 1)); j++) {
        uint32_t w8[8];
        x.to_dev(w8);
        uint32_t* e = &loc[dir][LOCAL_WORDS * (off + j)];
        for (int q = 0; q < NL; q++) {  // the same limbs as Fr::unpack
          const int o = LB * q, i = o >> 5, sh = o & 31;
          const uint64_t pair = ((uint64_t)(i + 1 < 8 ? w8[i + 1] : 0u) << 32) | w8[i];
          e[q] = (uint32_t)(pair >> sh) & LMASK;
        }
        x = HFr::mul(x, wk);
      }
    }
  }
  // 2^-L and (g^(2^L) - 1)^-1 for every L
  std::vector<uint32_t> ninv(8 * (MAX_LOG + 1)), zinv(8 * (MAX_LOG + 1));
  {
    const HFr two_inv = HFr::inv(HFr::from_uint(2));
    HFr x = HFr::one();
    HFr gpow = five;  // g^(2^L)
    for (int L = 0; L <= MAX_LOG; L++) {
      x.to_dev(&ninv[8 * L]);
      x = HFr::mul(x, two_inv);
      HFr::inv(HFr::sub(gpow, HFr::one())).to_dev(&zinv[8 * L]);
      gpow = HFr::sqr(gpow);
    }
  }
  size_t total = 0;
  for (auto& v : tabs) total += v.size();
  total += loc[0].size() + loc[1].size() + ninv.size() + zinv.size();
  auto* dt = new DeviceTables();
  dt->buf.alloc(total * 4);
  uint32_t* base = dt->buf.get();
  size_t off = 0;
  const uint32_t* ptrs[10];
  for (int i = 0; i < 8; i++) {
    ZK_HIP(hipMemcpy(base + off, tabs[i].data(), tabs[i].size() * 4, hipMemcpyHostToDevice));
    ptrs[i] = base + off;
    off += tabs[i].size();
  }
  for (int dir = 0; dir < 2; dir++) {
    ZK_HIP(hipMemcpy(base + off, loc[dir].data(), loc[dir].size() * 4, hipMemcpyHostToDevice));
    ptrs[8 + dir] = base + off;
    off += loc[dir].size();
  }
  dt->t.w[0] = {ptrs[0], ptrs[1]};
  dt->t.w[1] = {ptrs[2], ptrs[3]};
  dt->t.g[0] = {ptrs[4], ptrs[5]};
  dt->t.g[1] = {ptrs[6], ptrs[7]};
  dt->t.local[0] = ptrs[8];
  dt->t.local[1] = ptrs[9];
  ZK_HIP(hipMemcpy(base + off, ninv.data(), ninv.size() * 4, hipMemcpyHostToDevice));
  dt->t.ninv = base + off;
  off += ninv.size();
  ZK_HIP(hipMemcpy(base + off, zinv.data(), zinv.size() * 4, hipMemcpyHostToDevice));
  dt->t.coset_zinv = base + off;
  off += zinv.size();
  return dt;
}

}  // namespace

const NttTables& ntt_tables(int device) {
  static std::mutex mu;
  static std::map<int, DeviceTables*> cache;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(device);
  if (it != cache.end()) return it->second->t;
  DeviceTables* dt = build_tables();
  cache[device] = dt;
  return dt->t;
}

namespace {

// Per-pass twiddle tables (32 B per entry, M entries), built on first use for
// passes of M <= 2^TW_TABLE_MAX_LOG points and kept for the process: one
// multiplication per twiddled element instead of a power-table product.
constexpr int TW_TABLE_MAX_LOG = 24;

// A device table of 2^log_n entries made by `build` on first use and kept for
// the process (null when the stream is being captured, or out of memory: the
// callers then compute the factors instead).
template <class Build>
const uint32_t* cached_table(int kind, int a, int b, int log_n, hipStream_t st, Build&& build) {
  static std::mutex mu;
  static std::map<std::tuple<int, int, int, int>, DevBuf*> cache;
  const int dev = current_device();
  std::lock_guard<std::mutex> lock(mu);
  const auto key = std::make_tuple(dev, kind, a, b);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second->get();
  // not while the stream is being captured into a graph (the build waits)
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  ZK_HIP(hipStreamIsCapturing(st, &cs));
  if (cs != hipStreamCaptureStatusNone) return nullptr;
  auto* buf = new DevBuf();
  try {
    buf->alloc((size_t)32 << log_n);
  } catch (const Error&) {
    delete buf;
    return nullptr;
  }
  build(buf->get());
  ZK_HIP(hipGetLastError());
  // complete before any other stream can find it in the cache
  ZK_HIP(hipStreamSynchronize(st));
  cache[key] = buf;
  return buf->get();
}

const uint32_t* twiddle_table(int dir, int log_m, int k, const NttTables& T, hipStream_t st) {
  if (log_m > TW_TABLE_MAX_LOG || log_m <= k) return nullptr;
  return cached_table(0, dir, log_m * 32 + k, log_m, st, [&](uint32_t* out) {
    hipLaunchKernelGGL(k_twiddle_table, dim3(cdiv(1ull << log_m, 256)), dim3(256), 0, st, out, log_m, k, dir, T);
  });
}

// g^(+-bitrev(a)) / N by address a, for the quotient's coset scalings.
const uint32_t* coset_table(int dir, int log_n, const NttTables& T, hipStream_t st) {
  if (log_n > TW_TABLE_MAX_LOG) return nullptr;
  return cached_table(1, dir, log_n, log_n, st, [&](uint32_t* out) {
    hipLaunchKernelGGL(k_coset_table, dim3(cdiv(1ull << log_n, 256)), dim3(256), 0, st, out, log_n, dir, T);
  });
}

// The passes of one transform: pass j covers bits [log_m[j] - k[j], log_m[j])
// of the address (DIF order: the top bit range first).
struct PassPlan {
  int L = 0, kmax = 0, npass = 0;
  int k[NTT_MAX_LOG + 1] = {};
  int log_m[NTT_MAX_LOG + 1] = {};
  int log_g(int j) const {
    const int a = kmax - k[j], b = L - k[j];
    return a < b ? a : b;
  }
};

PassPlan plan_passes(int L, int min_pass, int max_k) {
  PassPlan pl;
  pl.L = L;
  // small transforms use 256-element workgroups so that a pass still spreads
  // over the device; large ones use 1024 (fewer passes over HBM)
  const int tk = tuning().ntt_kmax[L].load();
  pl.kmax = (tk >= 1 && tk <= NTT_MAX_K) ? tk : (L <= 18 ? 8 : NTT_MAX_K);
  int np = L == 0 ? 1 : (L + pl.kmax - 1) / pl.kmax;
  if (np < min_pass) np = min_pass;
  while ((L + np - 1) / np > max_k) np++;
  pl.npass = np;
  int lm = L;
  for (int j = 0; j < np; j++) {
    pl.k[j] = L / np + (j < L % np ? 1 : 0);
    pl.log_m[j] = lm;
    lm -= pl.k[j];
  }
  return pl;
}

// The passes of the quotient chain: a top pass of at most 2^7 points, so that
// the fused top kernel holds three regions of 2^9 elements in LDS and still
// reads runs of at least four consecutive elements (128 bytes) per group, and
// the other bits split evenly over passes of at most 2^10 points.
PassPlan plan_quotient(int L) {
  PassPlan pl = plan_passes(L, 1, NTT_MAX_K);  // the tuned or default tile size
  const int ktop = std::min(TOP_MAX_K - 2, L / 2);
  const int rest = L - ktop;
  const int nrest = (rest + NTT_MAX_K - 1) / NTT_MAX_K;
  pl.npass = 1 + nrest;
  pl.k[0] = ktop;
  pl.log_m[0] = L;
  int lm = L - ktop;
  for (int j = 1; j < pl.npass; j++) {
    pl.k[j] = rest / nrest + (j - 1 < rest % nrest ? 1 : 0);
    pl.log_m[j] = lm;
    lm -= pl.k[j];
  }
  // every pass has at least one group per block, the top pass four
  for (int j = 0; j < pl.npass; j++) pl.kmax = std::max(pl.kmax, pl.k[j]);
  pl.kmax = std::min(NTT_MAX_K, std::max(pl.kmax, ktop + 2));
  return pl;
}

// One pass of a transform over nvec vectors (direct pointers or a device table).
void launch_pass(uint32_t* const* data, uint32_t* const* dev_table, int nvec, const PassPlan& pl, int j, bool dit,
                 bool inverse, bool first, bool last, const NttFuse& fuse, const NttTables& T, hipStream_t st) {
  const int L = pl.L, k = pl.k[j];
  PassParams p{};
  if (dev_table)
    p.table = dev_table;
  else
    for (int v = 0; v < nvec; v++) p.data[v] = data[v];
  p.log_n = L;
  p.log_m = pl.log_m[j];
  p.k = k;
  p.log_g = pl.log_g(j);
  p.dit = dit;
  p.inverse = inverse ? 1 : 0;
  p.twiddle = pl.log_m[j] > k;
  p.tw = p.twiddle ? twiddle_table(p.inverse, pl.log_m[j], k, T, st) : nullptr;
  p.first = first;
  p.last = last;
  p.pre_mont = fuse.in_canonical;
  p.pre_coset = fuse.pre_coset;
  p.pre_bitrev = fuse.pre_bitrev;
  p.pre_const = fuse.pre_const;
  p.post_canon = fuse.out_canonical;
  p.post_coset = fuse.post_coset;
  p.post_bitrev = fuse.post_bitrev;
  p.post_const = fuse.post_const;
  p.post_table = fuse.post_table;
  const unsigned grid = 1u << (L - k - p.log_g);
  const size_t lds = (size_t)(1u << (k + p.log_g)) * NL * 4;
  unsigned threads = (1u << (k + p.log_g)) / 2;
  if (threads < 64) threads = 64;
  ProfScope ps("ntt_pass", st, (double)nvec * (double)(1ull << L) * k / 2.0);  // radix-2 butterflies
  hipLaunchKernelGGL(k_ntt_pass, dim3(grid, nvec), dim3(threads), lds, st, p, T);
  ZK_HIP(hipGetLastError());
}

void ntt_launch_impl(uint32_t* const* data, int nvec, int log_n, bool dit, bool inverse, const NttFuse& fuse,
                     hipStream_t st) {
  ZK_REQUIRE(log_n >= 0 && log_n <= MAX_LOG, "log_n out of range");
  ZK_REQUIRE(nvec >= 1 && nvec <= NTT_MAX_BATCH, "NTT batch size out of range");
  const NttTables& T = ntt_tables(current_device());
  const PassPlan pl = plan_passes(log_n, 1, NTT_MAX_K);
  for (int step = 0; step < pl.npass; step++) {
    const int j = dit ? (pl.npass - 1 - step) : step;
    launch_pass(data, nullptr, nvec, pl, j, dit, inverse, step == 0, step == pl.npass - 1, fuse, T, st);
  }
}

}  // namespace

void ntt_launch_batch(uint32_t* const* data, int nvec, int log_n, bool dit, bool inverse, const NttFuse& fuse,
                      hipStream_t st) {
  ntt_launch_impl(data, nvec, log_n, dit, inverse, fuse, st);
}

void ntt_launch(uint32_t* data, int log_n, bool dit, bool inverse, const NttFuse& fuse, hipStream_t st) {
  ntt_launch_batch(&data, 1, log_n, dit, inverse, fuse, st);
}

void qap_quotient_launch(uint32_t* const* abc, uint32_t* const* dev_table, int nproofs, int log_n, hipStream_t st,
                         hipEvent_t done_ev) {
  ZK_REQUIRE(log_n >= 2 && log_n <= MAX_LOG, "quotient domain out of range");
  ZK_REQUIRE(nproofs >= 1 && 3 * nproofs <= 65535 && (dev_table || nproofs == 1), "quotient batch out of range");
  const NttTables& T = ntt_tables(current_device());
  const int L = log_n;
  // at least two passes (the fused kernels need distinct top and bottom bit
  // ranges); the top pass keeps three 2^k-element regions in 64 KiB of LDS
  const PassPlan pl = plan_quotient(L);
  const int P = pl.npass;
  const int nvec = 3 * nproofs;
  NttFuse f1;
  f1.in_canonical = true;
  const NttFuse none;
  // inverse transform (DIF), all passes but the bottom one
  for (int j = 0; j < P - 1; j++) launch_pass(abc, dev_table, nvec, pl, j, false, true, j == 0, false, f1, T, st);
  FusedParams fp{};
  if (dev_table)
    fp.table = dev_table;
  else
    for (int v = 0; v < 3; v++) fp.data[v] = abc[v];
  fp.log_n = L;
  fp.ninv = T.ninv + 8 * L;
  fp.zinv = T.coset_zinv + 8 * L;
  fp.coset = coset_table(0, L, T, st);
  {
    // bottom: inverse DIF pass, coset scaling, forward DIT pass
    const int j = P - 1;
    fp.k = pl.k[j];
    fp.log_g = pl.log_g(j);
    const uint32_t E = 1u << (fp.k + fp.log_g);
    ProfScope ps("ntt_fused_bottom", st, (double)nvec * (double)(1ull << L) * fp.k);
    hipLaunchKernelGGL(k_ntt_fused_bottom, dim3(1u << (L - fp.k - fp.log_g), nvec), dim3(E < 128 ? 64 : E / 2),
                       (size_t)E * NL * 4, st, fp, T);
    ZK_HIP(hipGetLastError());
  }
  // forward DIT passes between the bottom and the top
  for (int j = P - 2; j >= 1; j--) launch_pass(abc, dev_table, nvec, pl, j, true, false, false, false, none, T, st);
  {
    // top: forward DIT pass and the pointwise quotient
    fp.k = pl.k[0];
    fp.tw[0] = twiddle_table(0, L, fp.k, T, st);
    const int a = TOP_MAX_K - fp.k, b = pl.log_g(0);
    fp.log_g = a < b ? a : b;
    const uint32_t E = 1u << (fp.k + fp.log_g);
    ProfScope ps("ntt_fused_top", st, (double)nproofs * (double)(1ull << L) * (1.5 * fp.k + 1.0), true);
    hipEvent_t e0, e1;
    const bool timed = ps.bind_events(&e0, &e1);
    // one butterfly of each of the three regions per thread and stage
    const uint32_t threads = 3 * E / 2 < 64 ? 64 : (3 * E / 2 > NTT_THREADS ? NTT_THREADS : 3 * E / 2);
    launch_ev(e0, timed ? e1 : done_ev, k_ntt_fused_top, dim3(1u << (L - fp.k - fp.log_g), nproofs), dim3(threads),
              (uint32_t)(3 * E * NL * 4), st, fp, T);
    ZK_HIP(hipGetLastError());
    if (timed && done_ev) ZK_HIP(hipEventRecord(done_ev, st));
  }
}

void bitrev_launch(uint32_t* data, int log_n, hipStream_t st) {
  if (log_n < 2) return;
  const uint32_t n = 1u << log_n;
  hipLaunchKernelGGL(k_bitrev, dim3(cdiv(n, 256)), dim3(256), 0, st, data, log_n, n);
  ZK_HIP(hipGetLastError());
}

}  // namespace zkvc
