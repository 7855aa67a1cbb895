// Number-theoretic transforms over Fr (the QAP's domain of 2^L points).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "field.hpp"

namespace zkvc {

constexpr int NTT_POW_BITS = 14;  // two-level power tables: 2^14 + 2^14 entries
constexpr int NTT_MAX_LOG = 28;
constexpr int NTT_MAX_BATCH = 3;  // vectors transformed together by one launch

// Two-level power tables for a fixed base b: b^x = lo[x & 0x3fff] * hi[x >> 14]
// for x < 2^28, elements in device Montgomery form (8 words each).
struct PowTable {
  const uint32_t* lo;
  const uint32_t* hi;
};

// Device-resident constants for every transform size up to 2^28.
struct NttTables {
  PowTable w[2];      // powers of omega_{2^28} (index 0) and of its inverse (index 1)
  PowTable g[2];      // powers of the coset shift g = 5 and of g^-1
  const uint32_t* local[2];  // omega_{2^k}^j for k = 1..10, j < 2^(k-1), at entry 2^(k-1) - 1 + j (12 words: 9 limbs)
  const uint32_t* ninv;      // 2^-L for L = 0..28 (8 words each)
  const uint32_t* coset_zinv; // (g^(2^L) - 1)^-1 for L = 0..28: 1/t on the coset g H
};

// Options fused into the first and last pass.
struct NttFuse {
  bool in_canonical = false;   // input elements are canonical integers (convert to Montgomery)
  bool out_canonical = false;  // write canonical integers
  int pre_coset = 0;           // multiply input element of index i by g^(+1 / -1 * i) before
  bool pre_bitrev = false;     //   ... where i = bitrev(address) if set, else the address
  const uint32_t* pre_const = nullptr;  // optional extra factor on the input (8 words, Montgomery)
  int post_coset = 0;          // multiply output element of index i by g^(+-i) after
  bool post_bitrev = false;    //   ... where i = bitrev(address) if set
  const uint32_t* post_const = nullptr; // optional extra factor on the output
  const uint32_t* post_table = nullptr; // if set, replaces post_coset and post_const: output element at
                                        //   address a times entry a (8 words, Montgomery)
};

const NttTables& ntt_tables(int device);

// base^x for x < 2^28 from a two-level table (one multiplication)
__device__ __forceinline__ Fr pow_lookup(const PowTable& t, uint32_t x) {
  const Fr a = Fr::load(t.lo + 8u * (x & ((1u << NTT_POW_BITS) - 1u)));
  const Fr b = Fr::load(t.hi + 8u * (x >> NTT_POW_BITS));
  return Fr::mul(a, b);
}

__device__ __forceinline__ uint32_t bitrev_bits(uint32_t a, int bits) {
  return bits == 0 ? 0u : (__builtin_bitreverse32(a) >> (32 - bits));
}

// In-place transform of n = 2^log_n Fr elements (8 words each, device Montgomery
// form unless fused conversions say otherwise).
//   dit = false: decimation in frequency, natural-order input -> bit-reversed output
//   dit = true : decimation in time, bit-reversed input -> natural-order output
//   inverse    : use omega^-1 (no 1/N scaling here; pass it as pre/post_const)
void ntt_launch(uint32_t* data, int log_n, bool dit, bool inverse, const NttFuse& fuse, hipStream_t st);
// The same transform applied to nvec <= NTT_MAX_BATCH vectors of the same size
// in one set of launches (more workgroups in flight per pass).
void ntt_launch_batch(uint32_t* const* data, int nvec, int log_n, bool dit, bool inverse, const NttFuse& fuse,
                      hipStream_t st);

// The QAP quotient of nproofs proofs of one domain size N = 2^log_n (>= 4):
// A, B, C hold canonical evaluations on the domain; afterwards A holds
// h = (A B - C) / Z on the coset g H: entry a is h(g omega_N^a) (natural
// order, device Montgomery form, a lazy value in [0, 2r)); B and C are
// clobbered.  The vectors are abc[0..2] (one proof) or, for any number of
// proofs, a device table of 3 nproofs entries: (A, B, C) per proof.  Same
// arithmetic as the chain iNTT / coset NTT / pointwise with ntt_launch_*,
// with the bottom and top passes of neighbouring transforms fused.
// done_ev, when not null, is bound to the last kernel's dispatch (it completes
// with it; eager streams only).
void qap_quotient_launch(uint32_t* const* abc, uint32_t* const* dev_table, int nproofs, int log_n, hipStream_t st,
                         hipEvent_t done_ev = nullptr);

// In-place bit-reversal permutation of 2^log_n elements.
void bitrev_launch(uint32_t* data, int log_n, hipStream_t st);

}  // namespace zkvc
