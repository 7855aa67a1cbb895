// Device arithmetic for the BN254 base field Fq and scalar field Fr.
//
// Representation.  A field element is held in registers as 9 limbs of 29 bits
// (261 bits) in Montgomery form with R = 2^261.  In memory it is stored packed
// as 8 little-endian 32-bit words (32 bytes), so arrays stay 32-byte aligned
// and an element moves with two 16-byte loads.
//
// Why 29-bit limbs on gfx950: v_mad_u64_u32 issues at full rate, as do 32-bit
// adds, so cost is the total VALU instruction count.  With 29-bit limbs every
// partial product is below 2^58 and a whole column (at most 18 products plus
// the incoming carry) fits a 64-bit accumulator.  Each partial product is then
// a single v_mad_u64_u32 into the accumulator with no per-product carry
// handling; carries are resolved once per column (Montgomery's reduction,
// 1985, in the column-interleaved "product scanning" order).
//
// Invariant: every Fp value returned by these functions is fully reduced,
// i.e. in [0, m) with each limb below 2^29.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "constants.hpp"

#define ZK_DEV __device__ __forceinline__

namespace zkvc {

constexpr int NL = 9;
constexpr int LB = 29;
constexpr uint32_t LMASK = (1u << LB) - 1u;

template <class M>
struct Fp;

// Out-of-line lazy Montgomery product and square (inputs and results in
// [0, 2m), see Fp::mul_core).  The G2 group law calls these
// instead of inlining ~230 instructions per product: an inlined G2 addition
// alone exceeds the instruction cache shared by two CUs (G1 additions fit, and
// run faster inlined).  The limbs travel as scalar arguments, so both
// operands and the result stay in VGPRs (an aggregate argument beyond the
// first would be passed through scratch).
template <class M>
__device__ __noinline__ Fp<M> fp_mul_call(uint32_t a0, uint32_t a1, uint32_t a2, uint32_t a3, uint32_t a4,
                                          uint32_t a5, uint32_t a6, uint32_t a7, uint32_t a8, uint32_t b0,
                                          uint32_t b1, uint32_t b2, uint32_t b3, uint32_t b4, uint32_t b5,
                                          uint32_t b6, uint32_t b7, uint32_t b8);
template <class M>
__device__ __noinline__ Fp<M> fp_sqr_call(uint32_t a0, uint32_t a1, uint32_t a2, uint32_t a3, uint32_t a4,
                                          uint32_t a5, uint32_t a6, uint32_t a7, uint32_t a8);

template <class M>
struct Fp {
  uint32_t v[NL];

  static ZK_DEV Fp zero() {
    Fp r;
#pragma unroll
    for (int k = 0; k < NL; k++) r.v[k] = 0u;
    return r;
  }
  static ZK_DEV Fp one() {  // R mod m: the Montgomery form of 1
    Fp r;
#pragma unroll
    for (int k = 0; k < NL; k++) r.v[k] = M::ONE[k];
    return r;
  }
  static ZK_DEV Fp raw_one() {  // the integer 1 (Montgomery form of R^-1)
    Fp r = zero();
    r.v[0] = 1u;
    return r;
  }

  // ---- packing between 8 x 32-bit words and 9 x 29-bit limbs ----
  static ZK_DEV Fp unpack(const uint32_t w[8]) {
    Fp r;
#pragma unroll
    for (int k = 0; k < NL; k++) {
      const int o = LB * k, q = o >> 5, sh = o & 31;
      const uint32_t lo = w[q];
      const uint32_t hi = (q + 1 < 8) ? w[q + 1] : 0u;
      r.v[k] = __builtin_amdgcn_alignbit(hi, lo, sh) & LMASK;
    }
    return r;
  }
  ZK_DEV void pack(uint32_t w[8]) const {
#pragma unroll
    for (int j = 0; j < 8; j++) {
      const int o = 32 * j, k = o / LB, sh = o % LB;
      uint64_t acc = (uint64_t)(v[k] >> sh);
      if (k + 1 < NL) acc |= (uint64_t)v[k + 1] << (LB - sh);
      if (k + 2 < NL && 2 * LB - sh < 32) acc |= (uint64_t)v[k + 2] << (2 * LB - sh);
      w[j] = (uint32_t)acc;
    }
  }
  static ZK_DEV Fp load(const uint32_t* p) {
    const uint4 a = reinterpret_cast<const uint4*>(p)[0];
    const uint4 b = reinterpret_cast<const uint4*>(p)[1];
    const uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
    return unpack(w);
  }
  ZK_DEV void store(uint32_t* p) const {
    uint32_t w[8];
    pack(w);
    reinterpret_cast<uint4*>(p)[0] = make_uint4(w[0], w[1], w[2], w[3]);
    reinterpret_cast<uint4*>(p)[1] = make_uint4(w[4], w[5], w[6], w[7]);
  }

  // ---- reduction helpers ----
  // r in [0, 2m) with r[8] possibly above 29 bits only by the value range -> [0, m)
  static ZK_DEV Fp reduce_once(const uint32_t r[NL]) {
    uint32_t d[NL];
    int32_t borrow = 0;
#pragma unroll
    for (int k = 0; k < NL; k++) {
      const int32_t t = (int32_t)r[k] - (int32_t)M::P[k] + borrow;
      d[k] = (uint32_t)t & LMASK;
      borrow = t >> LB;
    }
    Fp out;
    const bool keep = borrow < 0;
#pragma unroll
    for (int k = 0; k < NL; k++) out.v[k] = keep ? r[k] : d[k];
    return out;
  }

  // ---- ring operations ----
  static ZK_DEV Fp add(const Fp& a, const Fp& b) {
    uint32_t s[NL];
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < NL; k++) {
      const uint32_t t = a.v[k] + b.v[k] + c;
      s[k] = t & LMASK;
      c = t >> LB;
    }
    s[NL - 1] += c << LB;  // value < 2m < 2^255: the top limb absorbs the carry
    return reduce_once(s);
  }
  static ZK_DEV Fp sub(const Fp& a, const Fp& b) {
    uint32_t d[NL];
    int32_t borrow = 0;
#pragma unroll
    for (int k = 0; k < NL; k++) {
      const int32_t t = (int32_t)a.v[k] - (int32_t)b.v[k] + borrow;
      d[k] = (uint32_t)t & LMASK;
      borrow = t >> LB;
    }
    // if negative, add m back
    Fp out;
    uint32_t c = 0;
    const uint32_t mask = borrow < 0 ? 0xffffffffu : 0u;
#pragma unroll
    for (int k = 0; k < NL; k++) {
      const uint32_t t = d[k] + (M::P[k] & mask) + c;
      out.v[k] = t & LMASK;
      c = t >> LB;
    }
    return out;
  }
  static ZK_DEV Fp neg(const Fp& a) { return sub(zero(), a); }
  // m - a for a in [0, m), e.g. a stored coordinate: a representative in
  // (0, m] of -a with no conditional step (a lazy value for the group law)
  static ZK_DEV Fp neg_canon_lz(const Fp& a) {
    Fp out;
    int32_t borrow = 0;
#pragma unroll
    for (int k = 0; k < NL; k++) {
      const int32_t t = (int32_t)M::P[k] - (int32_t)a.v[k] + borrow;
      out.v[k] = (uint32_t)t & LMASK;
      borrow = t >> LB;
    }
    return out;
  }
  static ZK_DEV Fp dbl(const Fp& a) { return add(a, a); }

  // Montgomery product a*b*2^-261 mod m (column-interleaved reduction).
  static ZK_DEV Fp mul(const Fp& a, const Fp& b) {
    uint32_t r[NL];
    mul_core(a, b, r);
    return reduce_once(r);
  }
  // Squaring: off-diagonal products computed once against a doubled operand.
  static ZK_DEV Fp sqr(const Fp& a) {
    uint32_t r[NL];
    sqr_core(a, r);
    return reduce_once(r);
  }

  // The products before the final conditional subtraction: for inputs below
  // 2m the result is below m + 4m^2/2^261 < 2m (m < 2^254).
  static ZK_DEV void mul_core(const Fp& a, const Fp& b, uint32_t r[NL]) {
    uint64_t acc = 0;
    uint32_t m[NL];
#pragma unroll
    for (int k = 0; k < NL; k++) {
#pragma unroll
      for (int i = 0; i <= k; i++) acc += (uint64_t)a.v[i] * b.v[k - i];
#pragma unroll
      for (int i = 0; i < k; i++) acc += (uint64_t)m[i] * M::P[k - i];
      m[k] = ((uint32_t)acc * M::PINV) & LMASK;
      acc += (uint64_t)m[k] * M::P[0];
      acc >>= LB;
    }
#pragma unroll
    for (int k = NL; k < 2 * NL - 1; k++) {
#pragma unroll
      for (int i = k - NL + 1; i < NL; i++) acc += (uint64_t)a.v[i] * b.v[k - i];
#pragma unroll
      for (int i = k - NL + 1; i < NL; i++) acc += (uint64_t)m[i] * M::P[k - i];
      r[k - NL] = (uint32_t)acc & LMASK;
      acc >>= LB;
    }
    r[NL - 1] = (uint32_t)acc;
  }

  static ZK_DEV void sqr_core(const Fp& a, uint32_t r[NL]) {
    uint32_t a2[NL];
#pragma unroll
    for (int k = 0; k < NL; k++) a2[k] = a.v[k] << 1;  // < 2^30, products stay < 2^59
    uint64_t acc = 0;
    uint32_t m[NL];
#pragma unroll
    for (int k = 0; k < 2 * NL - 1; k++) {
      const int lo = k < NL ? 0 : k - NL + 1;
      const int hi = k < NL ? k : NL - 1;
#pragma unroll
      for (int i = lo; i <= hi; i++) {
        const int j = k - i;
        if (i < j) acc += (uint64_t)a2[i] * a.v[j];
        else if (i == j) acc += (uint64_t)a.v[i] * a.v[i];
      }
      if (k < NL) {
#pragma unroll
        for (int i = 0; i < k; i++) acc += (uint64_t)m[i] * M::P[k - i];
        m[k] = ((uint32_t)acc * M::PINV) & LMASK;
        acc += (uint64_t)m[k] * M::P[0];
      } else {
#pragma unroll
        for (int i = k - NL + 1; i < NL; i++) acc += (uint64_t)m[i] * M::P[k - i];
        r[k - NL] = (uint32_t)acc & LMASK;
      }
      acc >>= LB;
    }
    r[NL - 1] = (uint32_t)acc;
  }

  // ---- lazy forms for the group law: values kept in [0, 2m) ----
  // Products skip the final subtraction (see mul_core); sums and differences
  // fold back into [0, 2m) with 2m.  canon() returns the [0, m) representative.
  static ZK_DEV Fp reduce_2m(const uint32_t r[NL]) {  // [0, 4m) -> [0, 2m)
    uint32_t d[NL];
    int32_t borrow = 0;
#pragma unroll
    for (int k = 0; k < NL; k++) {
      const int32_t t = (int32_t)r[k] - (int32_t)M::P2[k] + borrow;
      d[k] = (uint32_t)t & LMASK;
      borrow = t >> LB;
    }
    Fp out;
    const bool keep = borrow < 0;
#pragma unroll
    for (int k = 0; k < NL; k++) out.v[k] = keep ? r[k] : d[k];
    return out;
  }
  static ZK_DEV Fp mul_lz(const Fp& a, const Fp& b) {
    Fp r;
    mul_core(a, b, r.v);
    return r;
  }
  static ZK_DEV Fp sqr_lz(const Fp& a) {
    Fp r;
    sqr_core(a, r.v);
    return r;
  }
  static ZK_DEV Fp add_lz(const Fp& a, const Fp& b) {
    uint32_t s[NL];
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < NL; k++) {
      const uint32_t t = a.v[k] + b.v[k] + c;
      s[k] = t & LMASK;
      c = t >> LB;
    }
    s[NL - 1] += c << LB;  // value < 4m < 2^256: the top limb absorbs the carry
    return reduce_2m(s);
  }
  static ZK_DEV Fp sub_lz(const Fp& a, const Fp& b) {
    uint32_t d[NL];
    int32_t borrow = 0;
#pragma unroll
    for (int k = 0; k < NL; k++) {
      const int32_t t = (int32_t)a.v[k] - (int32_t)b.v[k] + borrow;
      d[k] = (uint32_t)t & LMASK;
      borrow = t >> LB;
    }
    // if negative, add 2m back
    Fp out;
    uint32_t c = 0;
    const uint32_t mask = borrow < 0 ? 0xffffffffu : 0u;
#pragma unroll
    for (int k = 0; k < NL; k++) {
      const uint32_t t = d[k] + (M::P2[k] & mask) + c;
      out.v[k] = t & LMASK;
      c = t >> LB;
    }
    return out;
  }
  // a - b + 2m in (0, 4m) for a, b in [0, 2m), with no conditional step: an
  // operand of mul_lz, whose result stays below 2m for one operand below 4m
  // and the other below 2m (4m * 2m / 2^261 < m / 16).
  static ZK_DEV Fp sub_nr(const Fp& a, const Fp& b) {
    Fp out;
    int32_t borrow = 0;
#pragma unroll
    for (int k = 0; k < NL; k++) {
      const int32_t t = (int32_t)a.v[k] + (int32_t)M::P2[k] - (int32_t)b.v[k] + borrow;
      out.v[k] = (uint32_t)t & LMASK;
      borrow = t >> LB;
    }
    return out;  // the final borrow is 0: the value is positive
  }
  static ZK_DEV Fp canon(const Fp& a) { return reduce_once(a.v); }
  // a - b - 2c in [0, 2m) for a, b, c in [0, 2m): one pass forms
  // a + 6m - b - 2c in (0, 8m), then 4m and 2m are subtracted where they fit
  // (the x-coordinate of the addition formulas, in place of two lazy
  // subtractions and a doubling, each with its own conditional step).
  static ZK_DEV Fp sub3_lz(const Fp& a, const Fp& b, const Fp& c) {
    uint32_t t[NL];
    int32_t borrow = 0;
#pragma unroll
    for (int k = 0; k < NL; k++) {
      const int32_t x = (int32_t)a.v[k] + (int32_t)M::P6[k] - (int32_t)b.v[k] - (int32_t)(c.v[k] << 1) + borrow;
      t[k] = (uint32_t)x & LMASK;
      borrow = x >> LB;
    }
    // the value is positive and below 8m < 2^257, so the top limb ends with no borrow
    return cond_sub(cond_sub(t, M::P4).v, M::P2);
  }
  // r - s if that is not negative, else r
  static ZK_DEV Fp cond_sub(const uint32_t r[NL], const uint32_t s[NL]) {
    uint32_t d[NL];
    int32_t borrow = 0;
#pragma unroll
    for (int k = 0; k < NL; k++) {
      const int32_t x = (int32_t)r[k] - (int32_t)s[k] + borrow;
      d[k] = (uint32_t)x & LMASK;
      borrow = x >> LB;
    }
    Fp out;
    const bool keep = borrow < 0;
#pragma unroll
    for (int k = 0; k < NL; k++) out.v[k] = keep ? r[k] : d[k];
    return out;
  }
  // x = 0 (mod m) for x in [0, 4m) as sub_nr returns it.  x is then k*m with
  // k < 4, whose low limb takes one of four values: that screens out all but
  // about 2^-27 of the nonzero inputs before the exact test, which sits in a
  // branch of its own.
  static ZK_DEV bool is_zero_4m(const Fp& x) {
    const uint32_t l = x.v[0];
    // branch-free (compares of one value against constants become a search tree)
    const uint32_t t = min(min(l, l ^ M::P[0]), min(l ^ M::P2[0], l ^ ((M::P[0] + M::P2[0]) & LMASK)));
    if (t != 0u) return false;
    return is_zero(canon(reduce_2m(x.v)));
  }

  // lazy products through the out-of-line functions
  static ZK_DEV Fp mul_oop(const Fp& a, const Fp& b) {
    return fp_mul_call<M>(a.v[0], a.v[1], a.v[2], a.v[3], a.v[4], a.v[5], a.v[6], a.v[7], a.v[8], b.v[0], b.v[1],
                          b.v[2], b.v[3], b.v[4], b.v[5], b.v[6], b.v[7], b.v[8]);
  }
  static ZK_DEV Fp sqr_oop(const Fp& a) {
    return fp_sqr_call<M>(a.v[0], a.v[1], a.v[2], a.v[3], a.v[4], a.v[5], a.v[6], a.v[7], a.v[8]);
  }
  // the operations of the group law (curve.hpp): lazy, products inlined
  static ZK_DEV Fp cmul(const Fp& a, const Fp& b) { return mul_lz(a, b); }
  static ZK_DEV Fp csqr(const Fp& a) { return sqr_lz(a); }
  static ZK_DEV Fp cadd(const Fp& a, const Fp& b) { return add_lz(a, b); }
  static ZK_DEV Fp csub(const Fp& a, const Fp& b) { return sub_lz(a, b); }
  static ZK_DEV Fp cdbl(const Fp& a) { return add_lz(a, a); }
  static ZK_DEV Fp cneg(const Fp& a) { return sub_lz(zero(), a); }
  static ZK_DEV bool cis_zero(const Fp& a) { return is_zero(canon(a)); }
  // a difference whose only uses are products (and the zero test below):
  // a - b + 2m in (0, 4m), which the lazy product accepts (see sub_nr)
  static ZK_DEV Fp csub_p(const Fp& a, const Fp& b) { return sub_nr(a, b); }
  static ZK_DEV bool cis_zero_p(const Fp& a) { return is_zero_4m(a); }
  static ZK_DEV Fp csub3(const Fp& a, const Fp& b, const Fp& c) { return sub3_lz(a, b, c); }

  static ZK_DEV bool is_zero(const Fp& a) {
    uint32_t t = 0;
#pragma unroll
    for (int k = 0; k < NL; k++) t |= a.v[k];
    return t == 0u;
  }
  static ZK_DEV bool eq(const Fp& a, const Fp& b) {
    uint32_t t = 0;
#pragma unroll
    for (int k = 0; k < NL; k++) t |= a.v[k] ^ b.v[k];
    return t == 0u;
  }
  static ZK_DEV Fp select(bool c, const Fp& a, const Fp& b) {  // c ? a : b
    Fp r;
#pragma unroll
    for (int k = 0; k < NL; k++) r.v[k] = c ? a.v[k] : b.v[k];
    return r;
  }

  // canonical integer -> Montgomery form, and back
  static ZK_DEV Fp to_mont(const Fp& a) {
    Fp r2;
#pragma unroll
    for (int k = 0; k < NL; k++) r2.v[k] = M::R2[k];
    return mul(a, r2);
  }
  static ZK_DEV Fp from_mont(const Fp& a) { return mul(a, raw_one()); }

  // a^e for a small exponent held in 32-bit words, most significant first
  static ZK_DEV Fp pow_words(const Fp& a, const uint32_t* e, int nwords) {
    Fp r = one();
    for (int w = nwords - 1; w >= 0; w--) {
      for (int b = 31; b >= 0; b--) {
        r = sqr(r);
        if ((e[w] >> b) & 1u) r = mul(r, a);
      }
    }
    return r;
  }
  // inverse by Fermat's little theorem: a^(m-2); a must be nonzero
  static ZK_DEV Fp inv(const Fp& a) {
    uint32_t e[8];
#pragma unroll
    for (int k = 0; k < 8; k++) e[k] = M::P32[k];
    e[0] -= 2u;  // m is odd and > 2, no borrow
    return pow_words(a, e, 8);
  }
};

template <class M>
__device__ __noinline__ Fp<M> fp_mul_call(uint32_t a0, uint32_t a1, uint32_t a2, uint32_t a3, uint32_t a4,
                                          uint32_t a5, uint32_t a6, uint32_t a7, uint32_t a8, uint32_t b0,
                                          uint32_t b1, uint32_t b2, uint32_t b3, uint32_t b4, uint32_t b5,
                                          uint32_t b6, uint32_t b7, uint32_t b8) {
  const Fp<M> a{{a0, a1, a2, a3, a4, a5, a6, a7, a8}};
  const Fp<M> b{{b0, b1, b2, b3, b4, b5, b6, b7, b8}};
  return Fp<M>::mul_lz(a, b);
}
template <class M>
__device__ __noinline__ Fp<M> fp_sqr_call(uint32_t a0, uint32_t a1, uint32_t a2, uint32_t a3, uint32_t a4,
                                          uint32_t a5, uint32_t a6, uint32_t a7, uint32_t a8) {
  const Fp<M> a{{a0, a1, a2, a3, a4, a5, a6, a7, a8}};
  return Fp<M>::sqr_lz(a);
}

using Fq = Fp<FqParams>;
using Fr = Fp<FrParams>;

// Fq2 = Fq[i]/(i^2 + 1)
struct Fq2 {
  Fq c0, c1;
  static ZK_DEV Fq2 zero() { return {Fq::zero(), Fq::zero()}; }
  static ZK_DEV Fq2 one() { return {Fq::one(), Fq::zero()}; }
  static ZK_DEV Fq2 add(const Fq2& a, const Fq2& b) { return {Fq::add(a.c0, b.c0), Fq::add(a.c1, b.c1)}; }
  static ZK_DEV Fq2 sub(const Fq2& a, const Fq2& b) { return {Fq::sub(a.c0, b.c0), Fq::sub(a.c1, b.c1)}; }
  static ZK_DEV Fq2 dbl(const Fq2& a) { return {Fq::dbl(a.c0), Fq::dbl(a.c1)}; }
  static ZK_DEV Fq2 neg(const Fq2& a) { return {Fq::neg(a.c0), Fq::neg(a.c1)}; }
  static ZK_DEV Fq2 neg_canon_lz(const Fq2& a) { return {Fq::neg_canon_lz(a.c0), Fq::neg_canon_lz(a.c1)}; }
  // Karatsuba: 3 base multiplications
  static ZK_DEV Fq2 mul(const Fq2& a, const Fq2& b) {
    const Fq v0 = Fq::mul(a.c0, b.c0);
    const Fq v1 = Fq::mul(a.c1, b.c1);
    const Fq s = Fq::mul(Fq::add(a.c0, a.c1), Fq::add(b.c0, b.c1));
    return {Fq::sub(v0, v1), Fq::sub(Fq::sub(s, v0), v1)};
  }
  // (a0 + a1 i)^2 = (a0 + a1)(a0 - a1) + 2 a0 a1 i
  static ZK_DEV Fq2 sqr(const Fq2& a) {
    const Fq t = Fq::mul(a.c0, a.c1);
    return {Fq::mul(Fq::add(a.c0, a.c1), Fq::sub(a.c0, a.c1)), Fq::dbl(t)};
  }
  // the operations of the group law: lazy, through the out-of-line base-field products
  static ZK_DEV Fq2 cmul(const Fq2& a, const Fq2& b) {
    const Fq v0 = Fq::mul_oop(a.c0, b.c0);
    const Fq v1 = Fq::mul_oop(a.c1, b.c1);
    const Fq s = Fq::mul_oop(Fq::add_lz(a.c0, a.c1), Fq::add_lz(b.c0, b.c1));
    return {Fq::sub_lz(v0, v1), Fq::sub_lz(Fq::sub_lz(s, v0), v1)};
  }
  static ZK_DEV Fq2 csqr(const Fq2& a) {
    const Fq t = Fq::mul_oop(a.c0, a.c1);
    return {Fq::mul_oop(Fq::add_lz(a.c0, a.c1), Fq::sub_lz(a.c0, a.c1)), Fq::add_lz(t, t)};
  }
  static ZK_DEV Fq2 cadd(const Fq2& a, const Fq2& b) { return {Fq::add_lz(a.c0, b.c0), Fq::add_lz(a.c1, b.c1)}; }
  static ZK_DEV Fq2 csub(const Fq2& a, const Fq2& b) { return {Fq::sub_lz(a.c0, b.c0), Fq::sub_lz(a.c1, b.c1)}; }
  static ZK_DEV Fq2 cdbl(const Fq2& a) { return cadd(a, a); }
  static ZK_DEV Fq2 cneg(const Fq2& a) { return csub(zero(), a); }
  static ZK_DEV bool cis_zero(const Fq2& a) { return Fq::cis_zero(a.c0) && Fq::cis_zero(a.c1); }
  // differences feeding products keep the [0, 2m) range here: cmul and csqr
  // add and subtract their operands' components before multiplying
  static ZK_DEV Fq2 csub_p(const Fq2& a, const Fq2& b) { return csub(a, b); }
  static ZK_DEV Fq2 csub3(const Fq2& a, const Fq2& b, const Fq2& c) {
    return {Fq::sub3_lz(a.c0, b.c0, c.c0), Fq::sub3_lz(a.c1, b.c1, c.c1)};
  }
  static ZK_DEV bool cis_zero_p(const Fq2& a) { return cis_zero(a); }
  static ZK_DEV Fq2 canon(const Fq2& a) { return {Fq::canon(a.c0), Fq::canon(a.c1)}; }
  static ZK_DEV bool is_zero(const Fq2& a) { return Fq::is_zero(a.c0) && Fq::is_zero(a.c1); }
  static ZK_DEV bool eq(const Fq2& a, const Fq2& b) { return Fq::eq(a.c0, b.c0) && Fq::eq(a.c1, b.c1); }
  static ZK_DEV Fq2 select(bool c, const Fq2& a, const Fq2& b) {
    return {Fq::select(c, a.c0, b.c0), Fq::select(c, a.c1, b.c1)};
  }
  // 1/(a0 + a1 i) = (a0 - a1 i) / (a0^2 + a1^2)
  static ZK_DEV Fq2 inv(const Fq2& a) {
    const Fq d = Fq::inv(Fq::add(Fq::sqr(a.c0), Fq::sqr(a.c1)));
    return {Fq::mul(a.c0, d), Fq::neg(Fq::mul(a.c1, d))};
  }
  static ZK_DEV Fq2 load(const uint32_t* p) { return {Fq::load(p), Fq::load(p + 8)}; }
  ZK_DEV void store(uint32_t* p) const {
    c0.store(p);
    c1.store(p + 8);
  }
  static ZK_DEV Fq2 to_mont(const Fq2& a) { return {Fq::to_mont(a.c0), Fq::to_mont(a.c1)}; }
  static ZK_DEV Fq2 from_mont(const Fq2& a) { return {Fq::from_mont(a.c0), Fq::from_mont(a.c1)}; }
};

}  // namespace zkvc
