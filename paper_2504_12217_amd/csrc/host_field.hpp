// Host-side BN254 arithmetic: Fq, Fr (4 x 64-bit limbs, Montgomery R = 2^256),
// the tower Fq2 = Fq[i]/(i^2+1), Fq6 = Fq2[v]/(v^3 - xi), Fq12 = Fq6[w]/(w^2 - v)
// with xi = 9 + i, and Jacobian G1/G2 group operations.
//
// The host does the serial tails of the prover (Pippenger's window
// combination, the blinding terms of the proof, affine conversion) and the
// verifier's pairing.  These are chains of a few thousand dependent field
// operations: one CPU core runs them far faster than one GPU wavefront.
#pragma once
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "constants.hpp"

namespace zkvc {
namespace host {

typedef unsigned __int128 u128;

template <class M>
struct HF {
  uint64_t l[4];  // Montgomery form, fully reduced

  static HF zero() { return HF{{0, 0, 0, 0}}; }
  static HF one() { return HF{{M::ONE64[0], M::ONE64[1], M::ONE64[2], M::ONE64[3]}}; }

  static bool geq_mod(const uint64_t a[4]) {
    for (int k = 3; k >= 0; k--) {
      if (a[k] != M::P64[k]) return a[k] > M::P64[k];
    }
    return true;
  }
  static void sub_mod_inplace(uint64_t a[4]) {
    u128 borrow = 0;
    for (int k = 0; k < 4; k++) {
      u128 t = (u128)a[k] - M::P64[k] - borrow;
      a[k] = (uint64_t)t;
      borrow = (t >> 64) & 1;
    }
  }
  static HF add(const HF& a, const HF& b) {
    HF r;
    u128 c = 0;
    for (int k = 0; k < 4; k++) {
      c += (u128)a.l[k] + b.l[k];
      r.l[k] = (uint64_t)c;
      c >>= 64;
    }
    if (c || geq_mod(r.l)) sub_mod_inplace(r.l);
    return r;
  }
  static HF sub(const HF& a, const HF& b) {
    HF r;
    u128 borrow = 0;
    for (int k = 0; k < 4; k++) {
      u128 t = (u128)a.l[k] - b.l[k] - borrow;
      r.l[k] = (uint64_t)t;
      borrow = (t >> 64) & 1;
    }
    if (borrow) {
      u128 c = 0;
      for (int k = 0; k < 4; k++) {
        c += (u128)r.l[k] + M::P64[k];
        r.l[k] = (uint64_t)c;
        c >>= 64;
      }
    }
    return r;
  }
  static HF neg(const HF& a) { return sub(zero(), a); }
  static HF dbl(const HF& a) { return add(a, a); }
  // CIOS Montgomery multiplication (Koc, Acar, Kaliski 1996).  The modulus's
  // top word is below 2^63 - 1, so each row's two carry chains end within
  // four words (no fifth or sixth accumulator word) and the result is < 2m.
  static_assert(M::P64[3] < 0x7fffffffffffffffull, "modulus too wide for the short carry chain");
  static HF mul(const HF& a, const HF& b) {
    uint64_t t[4] = {0, 0, 0, 0};
    for (int i = 0; i < 4; i++) {
      u128 A = (u128)a.l[0] * b.l[i] + t[0];
      const uint64_t m = (uint64_t)A * M::PINV64;
      u128 C = ((u128)m * M::P64[0] + (uint64_t)A) >> 64;
      A >>= 64;
      for (int j = 1; j < 4; j++) {
        A += (u128)a.l[j] * b.l[i] + t[j];
        C += (u128)m * M::P64[j] + (uint64_t)A;
        A >>= 64;
        t[j - 1] = (uint64_t)C;
        C >>= 64;
      }
      t[3] = (uint64_t)(A + C);
    }
    HF r{{t[0], t[1], t[2], t[3]}};
    if (geq_mod(r.l)) sub_mod_inplace(r.l);
    return r;
  }
  static HF sqr(const HF& a) { return mul(a, a); }
  bool is_zero() const { return (l[0] | l[1] | l[2] | l[3]) == 0; }
  bool operator==(const HF& o) const { return std::memcmp(l, o.l, sizeof(l)) == 0; }
  bool operator!=(const HF& o) const { return !(*this == o); }

  // canonical little-endian words (value < m) <-> Montgomery
  static HF from_u64(const uint64_t c[4]) {
    HF a{{c[0], c[1], c[2], c[3]}};
    HF r2{{M::R2_64[0], M::R2_64[1], M::R2_64[2], M::R2_64[3]}};
    return mul(a, r2);
  }
  static HF from_u32(const uint32_t w[8]) {
    uint64_t c[4];
    for (int k = 0; k < 4; k++) c[k] = (uint64_t)w[2 * k] | ((uint64_t)w[2 * k + 1] << 32);
    return from_u64(c);
  }
  static HF from_uint(uint64_t v) {
    uint64_t c[4] = {v, 0, 0, 0};
    return from_u64(c);
  }
  void to_u64(uint64_t c[4]) const {
    HF one_raw{{1, 0, 0, 0}};
    HF r = mul(*this, one_raw);
    for (int k = 0; k < 4; k++) c[k] = r.l[k];
  }
  void to_u32(uint32_t w[8]) const {
    uint64_t c[4];
    to_u64(c);
    for (int k = 0; k < 4; k++) {
      w[2 * k] = (uint32_t)c[k];
      w[2 * k + 1] = (uint32_t)(c[k] >> 32);
    }
  }
  static bool canonical_ok(const uint32_t w[8]) {  // value < m
    uint64_t c[4];
    for (int k = 0; k < 4; k++) c[k] = (uint64_t)w[2 * k] | ((uint64_t)w[2 * k + 1] << 32);
    return !geq_mod(c);
  }
  // a^e, e as 4 little-endian 64-bit words
  static HF pow(const HF& a, const uint64_t e[4]) {
    HF r = one();
    for (int k = 3; k >= 0; k--)
      for (int b = 63; b >= 0; b--) {
        r = sqr(r);
        if ((e[k] >> b) & 1) r = mul(r, a);
      }
    return r;
  }
  // 1/a (0 for a = 0) by the binary extended Euclidean algorithm on the
  // stored integer A = a R (R = 2^256): it yields A^-1 = a^-1 R^-1, and two
  // products by R^2 give a^-1 R.  Runs of t zero bits are removed at once
  // (x / 2^t mod m as (x + k m) / 2^t with k = x (-m^-1) mod 2^t).
  static HF inv(const HF& a) {
    if (a.is_zero()) return zero();
    uint64_t u[4], v[4], x1[4] = {1, 0, 0, 0}, x2[4] = {0, 0, 0, 0};
    for (int k = 0; k < 4; k++) {
      u[k] = a.l[k];
      v[k] = M::P64[k];
    }
    auto is_one = [](const uint64_t* w) { return w[0] == 1 && (w[1] | w[2] | w[3]) == 0; };
    auto shr = [](uint64_t* w, int t) {  // 0 < t < 64
      for (int k = 0; k < 3; k++) w[k] = (w[k] >> t) | (w[k + 1] << (64 - t));
      w[3] >>= t;
    };
    // x / 2^t mod m for x in [0, m), 0 < t < 64: x + k m < 2^(256 + t) is exact in five words
    auto div_pow2 = [](uint64_t* x, int t) {
      const uint64_t k = (x[0] * M::PINV64) & ((1ull << t) - 1ull);
      u128 c = 0;
      for (int i = 0; i < 4; i++) {
        c += (u128)k * M::P64[i] + x[i];
        x[i] = (uint64_t)c;
        c >>= 64;
      }
      const uint64_t hi = (uint64_t)c;
      for (int i = 0; i < 3; i++) x[i] = (x[i] >> t) | (x[i + 1] << (64 - t));
      x[3] = (x[3] >> t) | (hi << (64 - t));
    };
    // strip the factors of two of w (nonzero), dividing x by the same power mod m
    auto strip = [&](uint64_t* w, uint64_t* x) {
      while ((w[0] & 1) == 0) {
        const int t = w[0] ? __builtin_ctzll(w[0]) : 63;
        shr(w, t);
        div_pow2(x, t);
      }
    };
    auto geq = [](const uint64_t* p, const uint64_t* q) {
      for (int k = 3; k >= 0; k--)
        if (p[k] != q[k]) return p[k] > q[k];
      return true;
    };
    auto sub_in = [](uint64_t* p, const uint64_t* q) {  // p -= q, p >= q
      u128 borrow = 0;
      for (int k = 0; k < 4; k++) {
        const u128 t = (u128)p[k] - q[k] - borrow;
        p[k] = (uint64_t)t;
        borrow = (t >> 64) & 1;
      }
    };
    auto sub_mod_in = [&](uint64_t* p, const uint64_t* q) {  // p = p - q mod m, both in [0, m)
      if (!geq(p, q)) {
        u128 c = 0;
        for (int k = 0; k < 4; k++) {  // p + m (below 2^255)
          c += (u128)p[k] + M::P64[k];
          p[k] = (uint64_t)c;
          c >>= 64;
        }
      }
      sub_in(p, q);
    };
    // invariants: x1 A = u, x2 A = v (mod m); u, v > 0 with gcd(u, v) = 1
    while (!is_one(u) && !is_one(v)) {
      strip(u, x1);
      strip(v, x2);
      if (is_one(u) || is_one(v)) break;
      if (geq(u, v)) {
        sub_in(u, v);
        sub_mod_in(x1, x2);
      } else {
        sub_in(v, u);
        sub_mod_in(x2, x1);
      }
    }
    HF r;
    for (int k = 0; k < 4; k++) r.l[k] = is_one(u) ? x1[k] : x2[k];
    const HF r2{{M::R2_64[0], M::R2_64[1], M::R2_64[2], M::R2_64[3]}};
    return mul(mul(r, r2), r2);
  }
  // a^(m-2), the inverse by Fermat's little theorem
  static HF inv_fermat(const HF& a) {
    uint64_t e[4] = {M::P64[0] - 2, M::P64[1], M::P64[2], M::P64[3]};
    return pow(a, e);
  }

  // Device representation: 8 words of x * 2^261 mod m.
  static const HF& dev_r() {  // Montgomery form of 2^261 mod m
    static const HF v = from_u64(M::DEVR_64);
    return v;
  }
  static const HF& dev_r_inv() {
    static const HF v = inv(dev_r());
    return v;
  }
  static HF from_dev(const uint32_t w[8]) { return mul(from_u32(w), dev_r_inv()); }
  void to_dev(uint32_t w[8]) const { mul(*this, dev_r()).to_u32(w); }
};

using HFq = HF<FqParams>;
using HFr = HF<FrParams>;

// ---------------------------------------------------------------- Fq2
struct HFq2 {
  HFq c0, c1;
  static HFq2 zero() { return {HFq::zero(), HFq::zero()}; }
  static HFq2 one() { return {HFq::one(), HFq::zero()}; }
  static HFq2 add(const HFq2& a, const HFq2& b) { return {HFq::add(a.c0, b.c0), HFq::add(a.c1, b.c1)}; }
  static HFq2 sub(const HFq2& a, const HFq2& b) { return {HFq::sub(a.c0, b.c0), HFq::sub(a.c1, b.c1)}; }
  static HFq2 neg(const HFq2& a) { return {HFq::neg(a.c0), HFq::neg(a.c1)}; }
  static HFq2 dbl(const HFq2& a) { return add(a, a); }
  static HFq2 mul(const HFq2& a, const HFq2& b) {
    HFq v0 = HFq::mul(a.c0, b.c0), v1 = HFq::mul(a.c1, b.c1);
    HFq s = HFq::mul(HFq::add(a.c0, a.c1), HFq::add(b.c0, b.c1));
    return {HFq::sub(v0, v1), HFq::sub(HFq::sub(s, v0), v1)};
  }
  static HFq2 sqr(const HFq2& a) { return mul(a, a); }
  static HFq2 scale(const HFq2& a, const HFq& k) { return {HFq::mul(a.c0, k), HFq::mul(a.c1, k)}; }
  static HFq2 conj(const HFq2& a) { return {a.c0, HFq::neg(a.c1)}; }
  static HFq2 inv(const HFq2& a) {
    HFq d = HFq::inv(HFq::add(HFq::sqr(a.c0), HFq::sqr(a.c1)));
    return {HFq::mul(a.c0, d), HFq::neg(HFq::mul(a.c1, d))};
  }
  // multiply by xi = 9 + i
  static HFq2 mul_xi(const HFq2& a) {
    HFq nine = HFq::from_uint(9);
    return {HFq::sub(HFq::mul(a.c0, nine), a.c1), HFq::add(HFq::mul(a.c1, nine), a.c0)};
  }
  bool is_zero() const { return c0.is_zero() && c1.is_zero(); }
  bool operator==(const HFq2& o) const { return c0 == o.c0 && c1 == o.c1; }
  bool operator!=(const HFq2& o) const { return !(*this == o); }
  static HFq2 pow(const HFq2& a, const uint64_t* e, int nwords) {
    HFq2 r = one();
    for (int k = nwords - 1; k >= 0; k--)
      for (int b = 63; b >= 0; b--) {
        r = sqr(r);
        if ((e[k] >> b) & 1) r = mul(r, a);
      }
    return r;
  }
};

// Width-5 non-adjacent form of a 256-bit k (little-endian words): digits
// d[i] in {0, +-1, +-3, ..., +-15}, k = sum_i d[i] 2^i, every nonzero digit
// followed by at least four zeros.  Returns the digit count (at most 257).
inline int wnaf5(const uint64_t k_in[4], int8_t d[260]) {
  uint64_t k[5] = {k_in[0], k_in[1], k_in[2], k_in[3], 0};
  int n = 0;
  while (k[0] | k[1] | k[2] | k[3] | k[4]) {
    int v = 0;
    if (k[0] & 1) {
      v = (int)(k[0] & 31);
      if (v >= 16) v -= 32;
      // k -= v, leaving k divisible by 32
      if (v > 0) {
        u128 t = (u128)k[0] - (uint64_t)v;
        k[0] = (uint64_t)t;
        for (int w = 1; w < 5 && (t >> 64); w++) {
          t = (u128)k[w] - 1;
          k[w] = (uint64_t)t;
        }
      } else {
        u128 t = (u128)k[0] + (uint64_t)(-v);
        k[0] = (uint64_t)t;
        for (int w = 1; w < 5 && (t >> 64); w++) {
          t = (u128)k[w] + 1;
          k[w] = (uint64_t)t;
        }
      }
    }
    d[n++] = (int8_t)v;
    for (int w = 0; w < 4; w++) k[w] = (k[w] >> 1) | (k[w + 1] << 63);
    k[4] >>= 1;
  }
  return n;
}

// ---------------------------------------------------------------- Jacobian points
// Generic over the coordinate field (HFq for G1, HFq2 for G2); a = 0.
template <class F>
struct Jac {
  F X, Y, Z;  // x = X/Z^2, y = Y/Z^3; Z = 0 is infinity
  static Jac inf() { return {F::one(), F::one(), F::zero()}; }
  bool is_inf() const { return Z.is_zero(); }
  static Jac from_affine(const F& x, const F& y) { return {x, y, F::one()}; }

  static Jac dbl(const Jac& p) {
    if (p.is_inf() || p.Y.is_zero()) return inf();
    F YY = F::sqr(p.Y);
    F S = F::dbl(F::dbl(F::mul(p.X, YY)));
    F XX = F::sqr(p.X);
    F M = F::add(F::dbl(XX), XX);
    F X3 = F::sub(F::sqr(M), F::dbl(S));
    F YYYY8 = F::dbl(F::dbl(F::dbl(F::sqr(YY))));
    F Y3 = F::sub(F::mul(M, F::sub(S, X3)), YYYY8);
    F Z3 = F::dbl(F::mul(p.Y, p.Z));
    return {X3, Y3, Z3};
  }
  static Jac add(const Jac& p, const Jac& q) {
    if (p.is_inf()) return q;
    if (q.is_inf()) return p;
    F Z1Z1 = F::sqr(p.Z), Z2Z2 = F::sqr(q.Z);
    F U1 = F::mul(p.X, Z2Z2), U2 = F::mul(q.X, Z1Z1);
    F S1 = F::mul(F::mul(p.Y, q.Z), Z2Z2), S2 = F::mul(F::mul(q.Y, p.Z), Z1Z1);
    if (U1 == U2) {
      if (S1 == S2) return dbl(p);
      return inf();
    }
    F H = F::sub(U2, U1), Rr = F::sub(S2, S1);
    F HH = F::sqr(H), HHH = F::mul(H, HH);
    F V = F::mul(U1, HH);
    F X3 = F::sub(F::sub(F::sqr(Rr), HHH), F::dbl(V));
    F Y3 = F::sub(F::mul(Rr, F::sub(V, X3)), F::mul(S1, HHH));
    F Z3 = F::mul(F::mul(p.Z, q.Z), H);
    return {X3, Y3, Z3};
  }
  static Jac neg(const Jac& p) { return {p.X, F::neg(p.Y), p.Z}; }
  // P + (x, y) with an affine second operand (Z2 = 1)
  static Jac add_affine(const Jac& p, const F& x2, const F& y2) {
    if (p.is_inf()) return from_affine(x2, y2);
    F Z1Z1 = F::sqr(p.Z);
    F U2 = F::mul(x2, Z1Z1);
    F S2 = F::mul(F::mul(y2, p.Z), Z1Z1);
    if (p.X == U2) {
      if (p.Y == S2) return dbl(p);
      return inf();
    }
    F H = F::sub(U2, p.X), Rr = F::sub(S2, p.Y);
    F HH = F::sqr(H), HHH = F::mul(H, HH);
    F V = F::mul(p.X, HH);
    F X3 = F::sub(F::sub(F::sqr(Rr), HHH), F::dbl(V));
    F Y3 = F::sub(F::mul(Rr, F::sub(V, X3)), F::mul(p.Y, HHH));
    return {X3, Y3, F::mul(p.Z, H)};
  }
  // scalar given as little-endian 64-bit words (4-bit fixed window)
  static Jac mul(const Jac& p, const uint64_t k[4]) {
    Jac table[16];
    table[0] = inf();
    for (int i = 1; i < 16; i++) table[i] = add(table[i - 1], p);
    Jac acc = inf();
    for (int w = 63; w >= 0; w--) {
      for (int d = 0; d < 4; d++) acc = dbl(acc);
      const int nib = (int)((k[w / 16] >> (4 * (w % 16))) & 15);
      if (nib) acc = add(acc, table[nib]);
    }
    return acc;
  }
  // t[i] = (2i + 1) P for i < 8
  static void odd_multiples(const Jac& p, Jac t[8]) {
    const Jac p2 = dbl(p);
    t[0] = p;
    for (int i = 1; i < 8; i++) t[i] = add(t[i - 1], p2);
  }
  // sum_j (+-k_j) P_j for n terms sharing one doubling chain (Straus), each
  // scalar in width-5 NAF over its odd multiples tab[j]; neg[j] negates term j
  static Jac naf_multi(int n, const Jac (*tab)[8], const uint64_t (*k)[4], const bool* neg) {
    int8_t d[4][260];
    int len[4], top = 0;
    for (int j = 0; j < n; j++) {
      len[j] = wnaf5(k[j], d[j]);
      top = len[j] > top ? len[j] : top;
    }
    Jac acc = inf();
    for (int i = top - 1; i >= 0; i--) {
      acc = dbl(acc);
      for (int j = 0; j < n; j++) {
        const int v = i < len[j] ? (neg[j] ? -d[j][i] : d[j][i]) : 0;
        if (v > 0) acc = add(acc, tab[j][v >> 1]);
        if (v < 0) acc = add(acc, Jac::neg(tab[j][(-v) >> 1]));
      }
    }
    return acc;
  }
  void to_affine(F& x, F& y) const {  // requires !is_inf()
    F zi = F::inv(Z);
    F zi2 = F::sqr(zi);
    x = F::mul(X, zi2);
    y = F::mul(Y, F::mul(zi2, zi));
  }
  bool eq(const Jac& q) const {
    if (is_inf() || q.is_inf()) return is_inf() && q.is_inf();
    F Z1Z1 = F::sqr(Z), Z2Z2 = F::sqr(q.Z);
    if (F::mul(X, Z2Z2) != F::mul(q.X, Z1Z1)) return false;
    return F::mul(F::mul(Y, q.Z), Z2Z2) == F::mul(F::mul(q.Y, Z), Z1Z1);
  }
};

using G1J = Jac<HFq>;
using G2J = Jac<HFq2>;

// ---------------------------------------------------------------- GLV on G1
// G1 has the endomorphism phi(x, y) = (beta x, y) with beta a primitive cube
// root of unity in Fq; on the order-r group phi is multiplication by a cube
// root of unity lambda in Fr (Gallant, Lambert and Vanstone, CRYPTO 2001).
// A scalar splits as k = k1 + k2 lambda (mod r) with |k1|, |k2| < 2^128, so
// k P = k1 P + k2 phi(P) takes half the doublings, and the two halves can run
// on two threads.
struct GlvSplit {
  uint64_t mag[2][4];  // |k1|, |k2|
  bool neg[2];         // k1 < 0, k2 < 0
};

namespace glv_detail {
// low 4 and high 4 words of the 512-bit product a b
inline void mul_256(const uint64_t a[4], const uint64_t b[4], uint64_t lo[4], uint64_t hi[4]) {
  uint64_t t[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int i = 0; i < 4; i++) {
    u128 c = 0;
    for (int j = 0; j < 4; j++) {
      c += (u128)a[i] * b[j] + t[i + j];
      t[i + j] = (uint64_t)c;
      c >>= 64;
    }
    t[i + 4] = (uint64_t)c;
  }
  for (int w = 0; w < 4; w++) {
    lo[w] = t[w];
    hi[w] = t[w + 4];
  }
}
inline void sub_256(uint64_t a[4], const uint64_t b[4]) {  // a -= b mod 2^256
  u128 borrow = 0;
  for (int w = 0; w < 4; w++) {
    const u128 t = (u128)a[w] - b[w] - borrow;
    a[w] = (uint64_t)t;
    borrow = (t >> 64) & 1;
  }
}
// two's complement value of a (mod 2^256) -> sign and magnitude
inline bool to_sign_mag(uint64_t a[4]) {
  if (!(a[3] >> 63)) return false;
  uint64_t m[4] = {0, 0, 0, 0};
  sub_256(m, a);
  for (int w = 0; w < 4; w++) a[w] = m[w];
  return true;
}
}  // namespace glv_detail

// k < r (little-endian words).  With the lattice basis v1 = (a1, -b1'),
// v2 = (a2, b2) of {(a, b): a + b lambda = 0 mod r}: c1 = floor(k g1 / 2^256),
// c2 = floor(k g2 / 2^256) approximate k b2 / r and k b1' / r, and
// (k1, k2) = (k, 0) - c1 v1 - c2 v2 lies in the lattice's coset of (k, 0),
// hence k1 + k2 lambda = k (mod r), with |k1| <= a1 + a2 and |k2| <= b1' + b2
// since both floors are off by less than one.
inline GlvSplit glv_split(const uint64_t k[4]) {
  using namespace glv_detail;
  uint64_t lo[4], c1[4], c2[4];
  mul_256(k, G1Glv::G1C, lo, c1);
  mul_256(k, G1Glv::G2C, lo, c2);
  GlvSplit s;
  uint64_t* k1 = s.mag[0];
  uint64_t* k2 = s.mag[1];
  for (int w = 0; w < 4; w++) k1[w] = k[w];
  uint64_t t[4], hi[4];
  mul_256(c1, G1Glv::A1, t, hi);
  sub_256(k1, t);
  mul_256(c2, G1Glv::A2, t, hi);
  sub_256(k1, t);
  mul_256(c1, G1Glv::B1ABS, k2, hi);
  mul_256(c2, G1Glv::B2, t, hi);
  sub_256(k2, t);
  s.neg[0] = to_sign_mag(k1);
  s.neg[1] = to_sign_mag(k2);
  return s;
}

inline G1J glv_phi(const G1J& p) {
  static const HFq beta = HFq::from_u64(G1Glv::BETA);
  return {HFq::mul(p.X, beta), p.Y, p.Z};
}

// One half of k P: half 0 is k1 P, half 1 is k2 phi(P).
inline G1J glv_half(const G1J& p, const GlvSplit& s, int half) {
  G1J tab[1][8];
  G1J::odd_multiples(half ? glv_phi(p) : p, tab[0]);
  return G1J::naf_multi(1, tab, &s.mag[half], &s.neg[half]);
}

// a P + b Q over one doubling chain of ~128 steps (four half-scalars)
inline G1J glv_mul2(const G1J& p, const uint64_t a[4], const G1J& q, const uint64_t b[4]) {
  const GlvSplit sa = glv_split(a), sb = glv_split(b);
  G1J tab[4][8];
  G1J::odd_multiples(p, tab[0]);
  G1J::odd_multiples(q, tab[2]);
  for (int i = 0; i < 8; i++) {
    tab[1][i] = glv_phi(tab[0][i]);
    tab[3][i] = glv_phi(tab[2][i]);
  }
  const uint64_t k[4][4] = {{sa.mag[0][0], sa.mag[0][1], sa.mag[0][2], sa.mag[0][3]},
                            {sa.mag[1][0], sa.mag[1][1], sa.mag[1][2], sa.mag[1][3]},
                            {sb.mag[0][0], sb.mag[0][1], sb.mag[0][2], sb.mag[0][3]},
                            {sb.mag[1][0], sb.mag[1][1], sb.mag[1][2], sb.mag[1][3]}};
  const bool neg[4] = {sa.neg[0], sa.neg[1], sb.neg[0], sb.neg[1]};
  return G1J::naf_multi(4, tab, k, neg);
}

// XYZZ (x = X/ZZ, y = Y/ZZZ, ZZ^3 = ZZZ^2) -> Jacobian without an inversion.
// Fixed-base table: entry [w][d] = d 2^(8w) P in affine form, for w < 32, d < 256;
// k P is then at most 32 mixed additions.
template <class F>
struct FixedBaseTable {
  std::vector<F> x, y;  // 32 * 256 entries; entry d = 0 unused
  void build(const Jac<F>& P) {
    const int total = 32 * 256;
    std::vector<Jac<F>> pts(total);
    Jac<F> base = P;
    for (int w = 0; w < 32; w++) {
      pts[w * 256] = Jac<F>::inf();
      for (int d = 1; d < 256; d++) pts[w * 256 + d] = Jac<F>::add(pts[w * 256 + d - 1], base);
      for (int k = 0; k < 8; k++) base = Jac<F>::dbl(base);
    }
    // simultaneous inversion of the Z coordinates
    std::vector<F> pre(total), zs(total);
    F acc = F::one();
    for (int i = 0; i < total; i++) {
      zs[i] = pts[i].is_inf() ? F::one() : pts[i].Z;
      pre[i] = acc;
      acc = F::mul(acc, zs[i]);
    }
    F inv = F::inv(acc);
    x.assign(total, F::zero());
    y.assign(total, F::zero());
    for (int i = total; i-- > 0;) {
      const F zi = F::mul(inv, pre[i]);
      inv = F::mul(inv, zs[i]);
      if (pts[i].is_inf()) continue;
      const F zi2 = F::sqr(zi);
      x[i] = F::mul(pts[i].X, zi2);
      y[i] = F::mul(pts[i].Y, F::mul(zi2, zi));
    }
  }
  bool empty() const { return x.empty(); }
  Jac<F> mul(const uint64_t k[4]) const {
    Jac<F> acc = Jac<F>::inf();
    for (int w = 0; w < 32; w++) {
      const int d = (int)((k[w / 8] >> (8 * (w % 8))) & 255);
      if (d) acc = Jac<F>::add_affine(acc, x[w * 256 + d], y[w * 256 + d]);
    }
    return acc;
  }
};

template <class F>
inline Jac<F> xyzz_to_jac(const F& X, const F& Y, const F& ZZ, const F& ZZZ) {
  if (ZZ.is_zero()) return Jac<F>::inf();
  // Let Z = ZZ * ZZZ.  Then Z^2 = ZZ^2 ZZZ^2 and x = X/ZZ = (X ZZ ZZZ^2)/Z^2;
  // Z^3 = ZZ^3 ZZZ^3 = ZZZ^2 ZZZ^3 (since ZZ^3 = ZZZ^2), so y = Y/ZZZ = (Y ZZZ^4)/Z^3.
  F Z = F::mul(ZZ, ZZZ);
  F ZZZ2 = F::sqr(ZZZ);
  F Xj = F::mul(F::mul(X, ZZ), ZZZ2);
  F Yj = F::mul(Y, F::sqr(ZZZ2));
  return {Xj, Yj, Z};
}

}  // namespace host
}  // namespace zkvc
