// Device group law for BN254 G1 (over Fq) and G2 (over Fq2, on the twist).
//
// Accumulators use XYZZ coordinates (X, Y, ZZ, ZZZ) with x = X/ZZ, y = Y/ZZZ
// and ZZ^3 = ZZZ^2; ZZ = 0 marks the point at infinity.  The addition and
// doubling formulas are the "add-2008-s", "madd-2008-s" and "dbl-2008-s-1"
// entries of Bernstein and Lange's Explicit-Formulas Database for a = 0:
// a mixed addition costs 8M + 2S and needs no inversion, which suits the
// bucket accumulation of Pippenger's method.  The coordinates are kept in
// the lazy range [0, 2m) (F::c* operations: no final subtraction after a
// product); products are inlined over Fq and out-of-line over Fq2 (keeping G2
// kernels inside the instruction cache).  Equality tests use the canonical
// representative; coordinates leave for the host through canonical stores.
//
// Infinity is exactly ZZ = 0 (every limb zero): inf() and the canonical
// stores write it that way, and no other value of ZZ is a multiple of m (ZZ
// of a sum is a product of nonzero factors; the exceptional cases of the
// formulas return inf() explicitly, and there are no points of order 2 to
// double), so is_inf needs no canonical reduction.
//
// Over Fq, differences whose only uses are products and a zero test
// (F::csub_p) skip the conditional step and lie in (0, 4m): the lazy product
// of operands below 4m is below m + 16m^2/2^261 < 2m.
//
// Affine points in memory are stored x then y (each coordinate 8 x 32-bit
// words in the device Montgomery form); the pair (0, 0) encodes infinity.
#pragma once
#include "field.hpp"

namespace zkvc {

template <class F>
struct Affine {
  F x, y;
};

template <class F>
struct Xyzz {
  F X, Y, ZZ, ZZZ;

  static ZK_DEV Xyzz inf() { return {F::one(), F::one(), F::zero(), F::zero()}; }
  static ZK_DEV bool is_inf(const Xyzz& p) { return F::is_zero(p.ZZ); }
  static ZK_DEV Xyzz from_affine(const Affine<F>& q) { return {q.x, q.y, F::one(), F::one()}; }

  // 2 * (x, y) for an affine input (mdbl-2008-s-1 with ZZ = ZZZ = 1)
  static ZK_DEV Xyzz dbl_affine(const Affine<F>& q) {
    if (F::cis_zero(q.y)) return inf();
    const F U = F::cdbl(q.y);
    const F V = F::csqr(U);
    const F W = F::cmul(U, V);
    const F S = F::cmul(q.x, V);
    const F xx = F::csqr(q.x);
    const F M = F::cadd(F::cdbl(xx), xx);
    const F X3 = F::csub(F::csqr(M), F::cdbl(S));
    const F Y3 = F::csub(F::cmul(M, F::csub(S, X3)), F::cmul(W, q.y));
    return {X3, Y3, V, W};
  }

  // 2P (dbl-2008-s-1)
  static ZK_DEV Xyzz dbl(const Xyzz& p) {
    if (is_inf(p) || F::cis_zero(p.Y)) return inf();
    const F U = F::cdbl(p.Y);
    const F V = F::csqr(U);
    const F W = F::cmul(U, V);
    const F S = F::cmul(p.X, V);
    const F xx = F::csqr(p.X);
    const F M = F::cadd(F::cdbl(xx), xx);
    const F X3 = F::csub(F::csqr(M), F::cdbl(S));
    const F Y3 = F::csub(F::cmul(M, F::csub(S, X3)), F::cmul(W, p.Y));
    return {X3, Y3, F::cmul(V, p.ZZ), F::cmul(W, p.ZZZ)};
  }

  // P + Q with Q affine (madd-2008-s), Q not infinity
  static ZK_DEV Xyzz madd(const Xyzz& p, const Affine<F>& q) {
    if (is_inf(p)) return from_affine(q);
    const F U2 = F::cmul(q.x, p.ZZ);
    const F S2 = F::cmul(q.y, p.ZZZ);
    const F P = F::csub_p(U2, p.X);
    const F R = F::csub_p(S2, p.Y);
    if (F::cis_zero_p(P)) {
      if (F::cis_zero_p(R)) return dbl_affine(q);
      return inf();
    }
    const F PP = F::csqr(P);
    const F PPP = F::cmul(P, PP);
    const F Q = F::cmul(p.X, PP);
    const F X3 = F::csub3(F::csqr(R), PPP, Q);
    const F Y3 = F::csub(F::cmul(R, F::csub_p(Q, X3)), F::cmul(p.Y, PPP));
    return {X3, Y3, F::cmul(p.ZZ, PP), F::cmul(p.ZZZ, PPP)};
  }

  // P + Q (add-2008-s)
  static ZK_DEV Xyzz add(const Xyzz& p, const Xyzz& q) {
    if (is_inf(p)) return q;
    if (is_inf(q)) return p;
    const F U1 = F::cmul(p.X, q.ZZ);
    const F U2 = F::cmul(q.X, p.ZZ);
    const F S1 = F::cmul(p.Y, q.ZZZ);
    const F S2 = F::cmul(q.Y, p.ZZZ);
    const F P = F::csub_p(U2, U1);
    const F R = F::csub_p(S2, S1);
    if (F::cis_zero_p(P)) {
      if (F::cis_zero_p(R)) return dbl(p);
      return inf();
    }
    const F PP = F::csqr(P);
    const F PPP = F::cmul(P, PP);
    const F Q = F::cmul(U1, PP);
    const F X3 = F::csub3(F::csqr(R), PPP, Q);
    const F Y3 = F::csub(F::cmul(R, F::csub_p(Q, X3)), F::cmul(S1, PPP));
    return {X3, Y3, F::cmul(F::cmul(p.ZZ, q.ZZ), PP), F::cmul(F::cmul(p.ZZZ, q.ZZZ), PPP)};
  }

  // the canonical representative of every coordinate (for values the host reads)
  static ZK_DEV Xyzz canon(const Xyzz& p) { return {F::canon(p.X), F::canon(p.Y), F::canon(p.ZZ), F::canon(p.ZZZ)}; }

  static ZK_DEV Xyzz neg(const Xyzz& p) { return {p.X, F::cneg(p.Y), p.ZZ, p.ZZZ}; }

  // [k]P for a small non-negative k (double-and-add, most significant bit first)
  static ZK_DEV Xyzz mul_small(const Xyzz& p, uint32_t k) {
    Xyzz acc = inf();
    if (k == 0u) return acc;
    const int top = 31 - __builtin_clz(k);
    acc = p;
    for (int b = top - 1; b >= 0; b--) {
      acc = dbl(acc);
      if ((k >> b) & 1u) acc = add(acc, p);
    }
    return acc;
  }
};

// ---------------------------------------------------------------- quad teams
// Latency-bound steps (reduction trees, buckets with few entries) leave most
// lanes idle while one addition's chain of dependent field products runs.
// There, four consecutive lanes (a quad) hold the same operands and compute
// one group operation together: per round each lane performs one of the
// formula's independent field products, and a DPP quad broadcast
// (quad_perm [k,k,k,k]) gives every lane all four results.  add-2008-s and
// madd-2008-s then take 4 rounds of one product instead of 12 + 2 and 8 + 2
// products in a chain.  Every branch inside is uniform over the quad (the
// operands are the same in all four lanes), so the four lanes stay active
// together, which the broadcast needs; the results are the same field
// elements as the serial formulas' (a square is the product x x).
// The broadcast stays a plain v_mov_b32_dpp: the empty asm statement takes
// its result as an operand, so the compiler cannot fold the DPP read into the
// instruction that consumes it (folded forms of the subtractions gave wrong
// results on gfx950).
template <int K>
ZK_DEV uint32_t quad_bcast_u32(uint32_t v) {
  uint32_t r = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, K * 0x55, 0xf, 0xf, false);
  asm volatile("" : "+v"(r));
  return r;
}
template <int K>
ZK_DEV Fq quad_bcast(const Fq& x) {
  Fq r;
#pragma unroll
  for (int q = 0; q < NL; q++) r.v[q] = quad_bcast_u32<K>(x.v[q]);
  return r;
}
template <int K>
ZK_DEV Fq2 quad_bcast(const Fq2& x) {
  return {quad_bcast<K>(x.c0), quad_bcast<K>(x.c1)};
}
template <class F>
ZK_DEV F sel4(uint32_t t, const F& a, const F& b, const F& c, const F& d) {
  const F ab = F::select(t & 1u, b, a), cd = F::select(t & 1u, d, c);
  return F::select(t & 2u, cd, ab);
}

template <class F>
struct QuadOps {
  using P = Xyzz<F>;
  // p + q; t = lane index in the quad (0..3); p and q equal in the four lanes
  static ZK_DEV P add(const P& p, const P& q, uint32_t t) {
    if (P::is_inf(p)) return q;
    if (P::is_inf(q)) return p;
    F r = F::cmul(sel4(t, p.X, q.X, p.Y, q.Y), sel4(t, q.ZZ, p.ZZ, q.ZZZ, p.ZZZ));
    const F U1 = quad_bcast<0>(r), U2 = quad_bcast<1>(r), S1 = quad_bcast<2>(r), S2 = quad_bcast<3>(r);
    const F Pd = F::csub_p(U2, U1), R = F::csub_p(S2, S1);
    if (F::cis_zero_p(Pd)) {
      if (F::cis_zero_p(R)) return P::dbl(p);
      return P::inf();
    }
    r = F::cmul(sel4(t, Pd, R, p.ZZ, p.ZZZ), sel4(t, Pd, R, q.ZZ, q.ZZZ));
    const F PP = quad_bcast<0>(r), RR = quad_bcast<1>(r), ZZ12 = quad_bcast<2>(r), ZZZ12 = quad_bcast<3>(r);
    r = F::cmul(sel4(t, Pd, U1, ZZ12, ZZ12), PP);
    const F PPP = quad_bcast<0>(r), Q = quad_bcast<1>(r), ZZ3 = quad_bcast<2>(r);
    const F X3 = F::csub3(RR, PPP, Q);
    r = F::cmul(sel4(t, R, S1, ZZZ12, ZZZ12), F::select(t == 0u, F::csub_p(Q, X3), PPP));
    const F T1 = quad_bcast<0>(r), T2 = quad_bcast<1>(r), ZZZ3 = quad_bcast<2>(r);
    return {X3, F::csub(T1, T2), ZZ3, ZZZ3};
  }
  // p + q with q affine, not infinity
  static ZK_DEV P madd(const P& p, const Affine<F>& q, uint32_t t) {
    if (P::is_inf(p)) return P::from_affine(q);
    const bool odd = t & 1u;
    F r = F::cmul(F::select(odd, q.y, q.x), F::select(odd, p.ZZZ, p.ZZ));
    const F U2 = quad_bcast<0>(r), S2 = quad_bcast<1>(r);
    const F Pd = F::csub_p(U2, p.X), R = F::csub_p(S2, p.Y);
    if (F::cis_zero_p(Pd)) {
      if (F::cis_zero_p(R)) return P::dbl_affine(q);
      return P::inf();
    }
    const F PR = F::select(odd, R, Pd);
    r = F::cmul(PR, PR);
    const F PP = quad_bcast<0>(r), RR = quad_bcast<1>(r);
    r = F::cmul(sel4(t, Pd, p.X, p.ZZ, p.ZZ), PP);
    const F PPP = quad_bcast<0>(r), Q = quad_bcast<1>(r), ZZ3 = quad_bcast<2>(r);
    const F X3 = F::csub3(RR, PPP, Q);
    r = F::cmul(sel4(t, R, p.Y, p.ZZZ, p.ZZZ), F::select(t == 0u, F::csub_p(Q, X3), PPP));
    const F T1 = quad_bcast<0>(r), T2 = quad_bcast<1>(r), ZZZ3 = quad_bcast<2>(r);
    return {X3, F::csub(T1, T2), ZZ3, ZZZ3};
  }
};

// Memory helpers: a G1 affine point is 16 words, a G2 affine point 32 words,
// an XYZZ accumulator 4 coordinates of the same widths.
template <class F>
struct PointIO;

template <>
struct PointIO<Fq> {
  static constexpr int AFF_WORDS = 16;
  static constexpr int XYZZ_WORDS = 32;
  static ZK_DEV Affine<Fq> load_affine(const uint32_t* p) { return {Fq::load(p), Fq::load(p + 8)}; }
  static ZK_DEV void store_affine(uint32_t* p, const Affine<Fq>& a) {
    a.x.store(p);
    a.y.store(p + 8);
  }
  static ZK_DEV bool affine_is_zero(const uint32_t* p) {
    const uint4* q = reinterpret_cast<const uint4*>(p);
    uint32_t t = 0;
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const uint4 v = q[k];
      t |= v.x | v.y | v.z | v.w;
    }
    return t == 0u;
  }
  static ZK_DEV Xyzz<Fq> load_xyzz(const uint32_t* p) {
    return {Fq::load(p), Fq::load(p + 8), Fq::load(p + 16), Fq::load(p + 24)};
  }
  static ZK_DEV void store_xyzz(uint32_t* p, const Xyzz<Fq>& a) {
    a.X.store(p);
    a.Y.store(p + 8);
    a.ZZ.store(p + 16);
    a.ZZZ.store(p + 24);
  }
};

template <>
struct PointIO<Fq2> {
  static constexpr int AFF_WORDS = 32;
  static constexpr int XYZZ_WORDS = 64;
  static ZK_DEV Affine<Fq2> load_affine(const uint32_t* p) { return {Fq2::load(p), Fq2::load(p + 16)}; }
  static ZK_DEV void store_affine(uint32_t* p, const Affine<Fq2>& a) {
    a.x.store(p);
    a.y.store(p + 16);
  }
  static ZK_DEV bool affine_is_zero(const uint32_t* p) {
    const uint4* q = reinterpret_cast<const uint4*>(p);
    uint32_t t = 0;
#pragma unroll
    for (int k = 0; k < 8; k++) {
      const uint4 v = q[k];
      t |= v.x | v.y | v.z | v.w;
    }
    return t == 0u;
  }
  static ZK_DEV Xyzz<Fq2> load_xyzz(const uint32_t* p) {
    return {Fq2::load(p), Fq2::load(p + 16), Fq2::load(p + 32), Fq2::load(p + 48)};
  }
  static ZK_DEV void store_xyzz(uint32_t* p, const Xyzz<Fq2>& a) {
    a.X.store(p);
    a.Y.store(p + 16);
    a.ZZ.store(p + 32);
    a.ZZZ.store(p + 48);
  }
};

}  // namespace zkvc
