// Groth16 verification on the host (Section II: Verify decides validity from
// the public parameters, the public input and the proof; Groth16 does so with
// a product of pairings).
//
// Pairing: optimal Ate on BN254 (Vercauteren 2010).  GT lives in the tower
// Fq2 = Fq[i]/(i^2+1), Fq6 = Fq2[v]/(v^3 - xi), Fq12 = Fq6[w]/(w^2 - v),
// xi = 9 + i, so that w^6 = xi.  A twist point (x, y) maps to E(Fq12) as
// (x w^2, y w^3).  The Miller loop runs over 6u + 2 with affine twist
// arithmetic, then adds pi(Q) and -pi^2(Q), where the Frobenius on the twist is
// (conj(x) xi^((p-1)/3), conj(y) xi^((p-1)/2)).  The final exponentiation is
// f^(p^6 - 1) (conjugate over inverse), then ^(p^2 + 1), then the hard part
// (p^4 - p^2 + 1)/r by square-and-multiply.
#include <cstring>
#include <vector>

#include "api_common.hpp"
#include "prover.hpp"

namespace zkvc {
namespace {

using host::HFq;
using host::HFq2;
using host::HFr;

struct F6 {
  HFq2 c0, c1, c2;
  static F6 zero() { return {HFq2::zero(), HFq2::zero(), HFq2::zero()}; }
  static F6 one() { return {HFq2::one(), HFq2::zero(), HFq2::zero()}; }
  static F6 add(const F6& a, const F6& b) { return {HFq2::add(a.c0, b.c0), HFq2::add(a.c1, b.c1), HFq2::add(a.c2, b.c2)}; }
  static F6 sub(const F6& a, const F6& b) { return {HFq2::sub(a.c0, b.c0), HFq2::sub(a.c1, b.c1), HFq2::sub(a.c2, b.c2)}; }
  static F6 neg(const F6& a) { return {HFq2::neg(a.c0), HFq2::neg(a.c1), HFq2::neg(a.c2)}; }
  static F6 mul(const F6& a, const F6& b) {
    // schoolbook with v^3 = xi
    const HFq2 a0b0 = HFq2::mul(a.c0, b.c0), a1b1 = HFq2::mul(a.c1, b.c1), a2b2 = HFq2::mul(a.c2, b.c2);
    const HFq2 cross12 = HFq2::add(HFq2::mul(a.c1, b.c2), HFq2::mul(a.c2, b.c1));
    const HFq2 cross01 = HFq2::add(HFq2::mul(a.c0, b.c1), HFq2::mul(a.c1, b.c0));
    const HFq2 cross02 = HFq2::add(HFq2::mul(a.c0, b.c2), HFq2::mul(a.c2, b.c0));
    return {HFq2::add(a0b0, HFq2::mul_xi(cross12)), HFq2::add(cross01, HFq2::mul_xi(a2b2)),
            HFq2::add(cross02, a1b1)};
  }
  static F6 mul_v(const F6& a) { return {HFq2::mul_xi(a.c2), a.c0, a.c1}; }
  static F6 inv(const F6& a) {
    const HFq2 t0 = HFq2::sub(HFq2::sqr(a.c0), HFq2::mul_xi(HFq2::mul(a.c1, a.c2)));
    const HFq2 t1 = HFq2::sub(HFq2::mul_xi(HFq2::sqr(a.c2)), HFq2::mul(a.c0, a.c1));
    const HFq2 t2 = HFq2::sub(HFq2::sqr(a.c1), HFq2::mul(a.c0, a.c2));
    const HFq2 det = HFq2::add(HFq2::mul(a.c0, t0),
                               HFq2::mul_xi(HFq2::add(HFq2::mul(a.c2, t1), HFq2::mul(a.c1, t2))));
    const HFq2 di = HFq2::inv(det);
    return {HFq2::mul(t0, di), HFq2::mul(t1, di), HFq2::mul(t2, di)};
  }
  bool is_zero() const { return c0.is_zero() && c1.is_zero() && c2.is_zero(); }
  bool operator==(const F6& o) const { return c0 == o.c0 && c1 == o.c1 && c2 == o.c2; }
};

struct F12 {
  F6 c0, c1;  // c0 + c1 w
  static F12 one() { return {F6::one(), F6::zero()}; }
  static F12 mul(const F12& a, const F12& b) {
    const F6 t0 = F6::mul(a.c0, b.c0), t1 = F6::mul(a.c1, b.c1);
    const F6 s = F6::mul(F6::add(a.c0, a.c1), F6::add(b.c0, b.c1));
    return {F6::add(t0, F6::mul_v(t1)), F6::sub(F6::sub(s, t0), t1)};
  }
  static F12 sqr(const F12& a) { return mul(a, a); }
  static F12 conj(const F12& a) { return {a.c0, F6::neg(a.c1)}; }
  static F12 inv(const F12& a) {
    // 1/(c0 + c1 w) = (c0 - c1 w)/(c0^2 - c1^2 v)
    const F6 d = F6::sub(F6::mul(a.c0, a.c0), F6::mul_v(F6::mul(a.c1, a.c1)));
    const F6 di = F6::inv(d);
    return {F6::mul(a.c0, di), F6::neg(F6::mul(a.c1, di))};
  }
  static F12 pow(const F12& a, const std::vector<uint64_t>& e) {
    F12 r = one();
    for (size_t k = e.size(); k-- > 0;)
      for (int b = 63; b >= 0; b--) {
        r = sqr(r);
        if ((e[k] >> b) & 1) r = mul(r, a);
      }
    return r;
  }
  bool is_one() const { return c0 == F6::one() && c1.is_zero(); }
};

// ---- multi-precision helpers for exponents (little-endian 64-bit words)
typedef unsigned __int128 u128;
std::vector<uint64_t> mp_mul(const std::vector<uint64_t>& a, const std::vector<uint64_t>& b) {
  std::vector<uint64_t> r(a.size() + b.size(), 0);
  for (size_t i = 0; i < a.size(); i++) {
    u128 c = 0;
    for (size_t j = 0; j < b.size(); j++) {
      c += (u128)a[i] * b[j] + r[i + j];
      r[i + j] = (uint64_t)c;
      c >>= 64;
    }
    r[i + b.size()] = (uint64_t)c;
  }
  while (r.size() > 1 && r.back() == 0) r.pop_back();
  return r;
}
std::vector<uint64_t> mp_add_small(std::vector<uint64_t> a, int64_t v) {  // a + v (v may be negative, result >= 0)
  if (v >= 0) {
    u128 c = (uint64_t)v;
    for (size_t i = 0; i < a.size() && c; i++) {
      c += a[i];
      a[i] = (uint64_t)c;
      c >>= 64;
    }
    if (c) a.push_back((uint64_t)c);
  } else {
    uint64_t borrow = (uint64_t)(-v);
    for (size_t i = 0; i < a.size() && borrow; i++) {
      const uint64_t t = a[i] - borrow;
      borrow = a[i] < borrow ? 1 : 0;
      a[i] = t;
    }
  }
  while (a.size() > 1 && a.back() == 0) a.pop_back();
  return a;
}
std::vector<uint64_t> mp_sub(std::vector<uint64_t> a, const std::vector<uint64_t>& b) {
  uint64_t borrow = 0;
  for (size_t i = 0; i < a.size(); i++) {
    const uint64_t bi = i < b.size() ? b[i] : 0;
    const u128 t = (u128)a[i] - bi - borrow;
    a[i] = (uint64_t)t;
    borrow = (uint64_t)((t >> 64) & 1);
  }
  while (a.size() > 1 && a.back() == 0) a.pop_back();
  return a;
}
// exact division by a multi-word divisor (schoolbook long division, bit by bit)
std::vector<uint64_t> mp_div_exact(const std::vector<uint64_t>& a, const std::vector<uint64_t>& d) {
  const size_t bits = a.size() * 64;
  std::vector<uint64_t> q(a.size(), 0), rem(d.size() + 1, 0);
  auto geq = [&](const std::vector<uint64_t>& x) {
    for (size_t i = x.size(); i-- > 0;) {
      const uint64_t di = i < d.size() ? d[i] : 0;
      if (x[i] != di) return x[i] > di;
    }
    return true;
  };
  for (size_t bit = bits; bit-- > 0;) {
    // rem = 2 rem + bit
    uint64_t carry = (a[bit / 64] >> (bit % 64)) & 1;
    for (auto& w : rem) {
      const uint64_t nc = w >> 63;
      w = (w << 1) | carry;
      carry = nc;
    }
    if (geq(rem)) {
      uint64_t borrow = 0;
      for (size_t i = 0; i < rem.size(); i++) {
        const uint64_t di = i < d.size() ? d[i] : 0;
        const u128 t = (u128)rem[i] - di - borrow;
        rem[i] = (uint64_t)t;
        borrow = (uint64_t)((t >> 64) & 1);
      }
      q[bit / 64] |= 1ull << (bit % 64);
    }
  }
  while (q.size() > 1 && q.back() == 0) q.pop_back();
  return q;
}

struct PairingConsts {
  HFq2 frob_x, frob_y;  // xi^((p-1)/3), xi^((p-1)/2)
  std::vector<uint64_t> hard, p_sq;
  unsigned __int128 ate;  // 6u + 2 (65 bits)
  PairingConsts() {
    const uint64_t u = 4965661367192848881ull;
    ate = (unsigned __int128)u * 6 + 2;
    std::vector<uint64_t> p(FqParams::P64, FqParams::P64 + 4), r(FrParams::P64, FrParams::P64 + 4);
    const std::vector<uint64_t> pm1 = mp_add_small(p, -1);
    // xi^((p-1)/3), xi^((p-1)/2)
    const std::vector<uint64_t> e3 = mp_div_exact(pm1, {3}), e2 = mp_div_exact(pm1, {2});
    const HFq2 xi = {HFq::from_uint(9), HFq::one()};
    frob_x = HFq2::pow(xi, e3.data(), (int)e3.size());
    frob_y = HFq2::pow(xi, e2.data(), (int)e2.size());
    p_sq = mp_mul(p, p);
    // (p^4 - p^2 + 1) / r
    const std::vector<uint64_t> p4 = mp_mul(p_sq, p_sq);
    hard = mp_div_exact(mp_add_small(mp_sub(p4, p_sq), 1), r);
  }
};

const PairingConsts& pc() {
  static const PairingConsts c;
  return c;
}

struct TwistPt {
  HFq2 x, y;
};

// line through T and Q (tangent if equal) evaluated at P = (xp, yp), as F12
F12 line_eval(const TwistPt& T, const TwistPt& Q, const HFq& xp, const HFq& yp, bool tangent) {
  HFq2 lam;
  if (tangent) {
    const HFq2 xx = HFq2::sqr(T.x);
    lam = HFq2::mul(HFq2::add(HFq2::dbl(xx), xx), HFq2::inv(HFq2::dbl(T.y)));
  } else {
    lam = HFq2::mul(HFq2::sub(Q.y, T.y), HFq2::inv(HFq2::sub(Q.x, T.x)));
  }
  F12 l;
  l.c0 = {HFq2{yp, HFq::zero()}, HFq2::zero(), HFq2::zero()};
  l.c1 = {HFq2::neg(HFq2::scale(lam, xp)), HFq2::sub(HFq2::mul(lam, T.x), T.y), HFq2::zero()};
  return l;
}

F12 vertical_eval(const TwistPt& T, const HFq& xp) {
  F12 l;
  l.c0 = {HFq2{xp, HFq::zero()}, HFq2::neg(T.x), HFq2::zero()};
  l.c1 = F6::zero();
  return l;
}

// affine twist arithmetic (no infinity handling needed inside the Miller loop)
TwistPt tw_dbl(const TwistPt& T) {
  const HFq2 xx = HFq2::sqr(T.x);
  const HFq2 lam = HFq2::mul(HFq2::add(HFq2::dbl(xx), xx), HFq2::inv(HFq2::dbl(T.y)));
  const HFq2 x3 = HFq2::sub(HFq2::sqr(lam), HFq2::dbl(T.x));
  return {x3, HFq2::sub(HFq2::mul(lam, HFq2::sub(T.x, x3)), T.y)};
}
TwistPt tw_add(const TwistPt& T, const TwistPt& Q) {
  const HFq2 lam = HFq2::mul(HFq2::sub(Q.y, T.y), HFq2::inv(HFq2::sub(Q.x, T.x)));
  const HFq2 x3 = HFq2::sub(HFq2::sub(HFq2::sqr(lam), T.x), Q.x);
  return {x3, HFq2::sub(HFq2::mul(lam, HFq2::sub(T.x, x3)), T.y)};
}

// f <- f * line(T, Q)(P); T <- T + Q (handles the coincident and opposite cases)
void step_add(F12& f, TwistPt& T, bool& T_inf, const TwistPt& Q, const HFq& xp, const HFq& yp) {
  if (T_inf) {
    T = Q;
    T_inf = false;
    return;
  }
  if (T.x == Q.x) {
    if (T.y == Q.y) {
      f = F12::mul(f, line_eval(T, T, xp, yp, true));
      T = tw_dbl(T);
    } else {
      f = F12::mul(f, vertical_eval(T, xp));
      T_inf = true;
    }
    return;
  }
  f = F12::mul(f, line_eval(T, Q, xp, yp, false));
  T = tw_add(T, Q);
}

F12 miller_loop(const HFq& xp, const HFq& yp, const TwistPt& Q) {
  const PairingConsts& c = pc();
  F12 f = F12::one();
  TwistPt T = Q;
  bool T_inf = false;
  int top = 127;
  while (!((c.ate >> top) & 1)) top--;
  for (int bit = top - 1; bit >= 0; bit--) {
    f = F12::sqr(f);
    if (!T_inf) {
      if (T.y.is_zero()) {
        f = F12::mul(f, vertical_eval(T, xp));
        T_inf = true;
      } else {
        f = F12::mul(f, line_eval(T, T, xp, yp, true));
        T = tw_dbl(T);
      }
    }
    if ((c.ate >> bit) & 1) step_add(f, T, T_inf, Q, xp, yp);
  }
  // Q1 = pi(Q), Q2 = -pi^2(Q)
  const TwistPt Q1 = {HFq2::mul(HFq2::conj(Q.x), c.frob_x), HFq2::mul(HFq2::conj(Q.y), c.frob_y)};
  const TwistPt P2 = {HFq2::mul(HFq2::conj(Q1.x), c.frob_x), HFq2::mul(HFq2::conj(Q1.y), c.frob_y)};
  const TwistPt Q2 = {P2.x, HFq2::neg(P2.y)};
  step_add(f, T, T_inf, Q1, xp, yp);
  step_add(f, T, T_inf, Q2, xp, yp);
  return f;
}

F12 final_exponentiation(const F12& f) {
  const PairingConsts& c = pc();
  F12 t = F12::mul(F12::conj(f), F12::inv(f));     // f^(p^6 - 1)
  t = F12::mul(F12::pow(t, c.p_sq), t);            // ^(p^2 + 1)
  return F12::pow(t, c.hard);                      // ^((p^4 - p^2 + 1)/r)
}

// ---- point decoding and checks
bool fq_from_words(const uint32_t w[8], HFq& out) {
  if (!HFq::canonical_ok(w)) return false;
  out = HFq::from_u32(w);
  return true;
}

struct G1A {
  bool inf = true;
  HFq x, y;
};
struct G2A {
  bool inf = true;
  HFq2 x, y;
};

bool decode_g1(const zkvc_g1& p, G1A& out) {
  bool zero = true;
  for (int k = 0; k < 8; k++) zero = zero && p.x[k] == 0 && p.y[k] == 0;
  if (zero) {
    out.inf = true;
    return true;
  }
  out.inf = false;
  return fq_from_words(p.x, out.x) && fq_from_words(p.y, out.y);
}
bool decode_g2(const zkvc_g2& p, G2A& out) {
  bool zero = true;
  for (int k = 0; k < 8; k++) zero = zero && p.x0[k] == 0 && p.x1[k] == 0 && p.y0[k] == 0 && p.y1[k] == 0;
  if (zero) {
    out.inf = true;
    return true;
  }
  out.inf = false;
  return fq_from_words(p.x0, out.x.c0) && fq_from_words(p.x1, out.x.c1) && fq_from_words(p.y0, out.y.c0) &&
         fq_from_words(p.y1, out.y.c1);
}
bool g1_on_curve(const G1A& p) {
  if (p.inf) return true;
  const HFq rhs = HFq::add(HFq::mul(HFq::sqr(p.x), p.x), HFq::from_uint(3));
  return HFq::sqr(p.y) == rhs;
}
const HFq2& twist_b() {
  static const HFq2 b = HFq2::mul(HFq2{HFq::from_uint(3), HFq::zero()}, HFq2::inv(HFq2{HFq::from_uint(9), HFq::one()}));
  return b;
}
bool g2_on_curve(const G2A& p) {
  if (p.inf) return true;
  const HFq2 rhs = HFq2::add(HFq2::mul(HFq2::sqr(p.x), p.x), twist_b());
  return HFq2::sqr(p.y) == rhs;
}
bool g2_in_subgroup(const G2A& p) {
  const host::G2J j = host::G2J::from_affine(p.x, p.y);
  uint64_t r[4] = {FrParams::P64[0], FrParams::P64[1], FrParams::P64[2], FrParams::P64[3]};
  return host::G2J::mul(j, r).is_inf();
}

// sum_i a_i P_i for small signed integer scalars (bucket method, 8-bit windows)
host::G1J small_msm(const std::vector<G1A>& pts, const std::vector<int64_t>& sc) {
  host::G1J total = host::G1J::inf();
  uint64_t maxabs = 0;
  for (int64_t v : sc) maxabs = std::max<uint64_t>(maxabs, (uint64_t)(v < 0 ? -v : v));
  int windows = 0;
  while (windows < 8 && (maxabs >> (8 * windows))) windows++;
  for (int w = windows - 1; w >= 0; w--) {
    for (int d = 0; d < 8; d++) total = host::G1J::dbl(total);
    std::vector<host::G1J> buckets(256, host::G1J::inf());
    for (size_t i = 0; i < pts.size(); i++) {
      if (pts[i].inf || sc[i] == 0) continue;
      const uint64_t mag = (uint64_t)(sc[i] < 0 ? -sc[i] : sc[i]);
      const uint32_t dgt = (uint32_t)((mag >> (8 * w)) & 255u);
      if (!dgt) continue;
      host::G1J P = host::G1J::from_affine(pts[i].x, sc[i] < 0 ? HFq::neg(pts[i].y) : pts[i].y);
      buckets[dgt] = host::G1J::add(buckets[dgt], P);
    }
    host::G1J run = host::G1J::inf(), acc = host::G1J::inf();
    for (int d = 255; d >= 1; d--) {
      run = host::G1J::add(run, buckets[d]);
      acc = host::G1J::add(acc, run);
    }
    total = host::G1J::add(total, acc);
  }
  return total;
}

}  // namespace

int groth16_verify(const uint8_t* vk, size_t vk_len, const int8_t* X, const int32_t* Y, const zkvc_proof* proof) {
  // ---- parse the key
  if (vk_len < 32 + 32 + 64 + 3 * 128 + 8 || std::memcmp(vk, "ZKVC-VK1", 8) != 0)
    throw Error(ZKVC_EFORMAT, "verification key: bad magic or length");
  uint32_t hdr[6];
  std::memcpy(hdr, vk + 8, sizeof(hdr));
  if (hdr[0] != 1) throw Error(ZKVC_EFORMAT, "verification key: unsupported version");
  Layout L;
  try {
    L = r1cs_layout(hdr[1], hdr[2], hdr[3], hdr[4]);
  } catch (const Error&) {
    throw Error(ZKVC_EFORMAT, "verification key: bad shape");
  }
  if ((uint32_t)L.log_n != hdr[5]) throw Error(ZKVC_EFORMAT, "verification key: domain size mismatch");
  size_t off = 32 + 32;
  zkvc_g1 a1;
  zkvc_g2 b2, g2, d2;
  std::memcpy(&a1, vk + off, 64);
  off += 64;
  std::memcpy(&b2, vk + off, 128);
  off += 128;
  std::memcpy(&g2, vk + off, 128);
  off += 128;
  std::memcpy(&d2, vk + off, 128);
  off += 128;
  uint64_t count;
  std::memcpy(&count, vk + off, 8);
  off += 8;
  if (count != L.ell + 1 || vk_len != off + 64 * count) throw Error(ZKVC_EFORMAT, "verification key: bad IC count");
  G1A alpha1;
  G2A beta2, gamma2, delta2;
  if (!decode_g1(a1, alpha1) || !decode_g2(b2, beta2) || !decode_g2(g2, gamma2) || !decode_g2(d2, delta2) ||
      !g1_on_curve(alpha1) || !g2_on_curve(beta2) || !g2_on_curve(gamma2) || !g2_on_curve(delta2))
    throw Error(ZKVC_EFORMAT, "verification key: point not on curve");
  std::vector<G1A> ic(count);
  for (uint64_t k = 0; k < count; k++) {
    zkvc_g1 p;
    std::memcpy(&p, vk + off + 64 * k, 64);
    if (!decode_g1(p, ic[k]) || !g1_on_curve(ic[k])) throw Error(ZKVC_EFORMAT, "verification key: IC off curve");
  }

  // ---- proof points: on the curve, not infinity, B in the order-r subgroup
  G1A A, C;
  G2A B;
  if (!decode_g1(proof->A, A) || !decode_g1(proof->C, C) || !decode_g2(proof->B, B)) return 0;
  if (A.inf || B.inf || C.inf) return 0;
  if (!g1_on_curve(A) || !g1_on_curve(C) || !g2_on_curve(B) || !g2_in_subgroup(B)) return 0;

  // ---- public-input combination: a_0 = 1, then x, then y
  std::vector<int64_t> sc(count);
  sc[0] = 1;
  const uint64_t an = (uint64_t)L.a * L.n, ab = (uint64_t)L.a * L.b;
  for (uint64_t i = 0; i < an; i++) sc[1 + i] = X[i];
  for (uint64_t i = 0; i < ab; i++) sc[1 + an + i] = Y[i];
  const host::G1J icsum = small_msm(ic, sc);

  // e(A, B) = e(alpha, beta) e(IC, gamma) e(C, delta)  <=>
  // e(A, B) e(-alpha, beta) e(-IC, gamma) e(-C, delta) = 1
  F12 f = miller_loop(A.x, A.y, {B.x, B.y});
  f = F12::mul(f, miller_loop(alpha1.x, HFq::neg(alpha1.y), {beta2.x, beta2.y}));
  if (!icsum.is_inf()) {
    HFq ix, iy;
    icsum.to_affine(ix, iy);
    f = F12::mul(f, miller_loop(ix, HFq::neg(iy), {gamma2.x, gamma2.y}));
  }
  f = F12::mul(f, miller_loop(C.x, HFq::neg(C.y), {delta2.x, delta2.y}));
  return final_exponentiation(f).is_one() ? 1 : 0;
}

}  // namespace zkvc
