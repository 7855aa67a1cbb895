"""Optimal-Ate pairing on BN254, written plainly for the CPU oracle.

TEST INFRASTRUCTURE ONLY (see oracle/bn254.py).

Groth16 verification decides validity with a product of pairings (Section II,
ZKP systems: Groth16 checks the QAP with elliptic-curve pairings).  This
module computes e: G1 x G2 -> GT by the textbook route, favouring plainness
over speed:

  * a G2 point on the twist E'(Fq2) is sent into E(Fq12) by the untwisting
    map (x, y) -> (x w^2, y w^3), where w^6 = 9 + i;
  * a Miller loop over the BN optimal-Ate parameter 6u + 2 evaluates chord
    and tangent lines through multiples of Q at P, all in E(Fq12) affine
    coordinates with Fq12 inversions;
  * the two Frobenius correction steps add pi(Q) and subtract pi^2(Q), where
    pi raises coordinates to the p-th power in Fq12 (done by exponentiation,
    with no precomputed Frobenius constants);
  * the final exponentiation raises the Miller value to (p^12 - 1)/r by
    plain square-and-multiply.

Raw GT values are not pinned to any external vector; the tests pin the map by
its defining properties (bilinearity, non-degeneracy, order r), and only the
boolean outcome of verification is used elsewhere.
"""
from .bn254 import (P, R, U, FQ12, ec_add, ec_double, ec_neg, f12_from_f2, f12_from_fq, f12_one,
                    f12_mul, f12_sqr, f12_pow, f12_sub, f12_inv, f12_scale, f12_is_one)

ATE_LOOP = 6 * U + 2
FINAL_EXP = (P**12 - 1) // R

_W = [0, 1] + [0] * 10          # w
_W2 = f12_mul(_W, _W)
_W3 = f12_mul(_W2, _W)


def untwist(q):
    """E'(Fq2) -> E(Fq12): (x, y) -> (x w^2, y w^3)."""
    if q is None:
        return None
    x, y = q
    return (f12_mul(f12_from_f2(x), _W2), f12_mul(f12_from_f2(y), _W3))


def embed_g1(p):
    if p is None:
        return None
    return (f12_from_fq(p[0]), f12_from_fq(p[1]))


def _line(t, q, p):
    """Value at p of the line through t and q (tangent if t == q); all in E(Fq12)."""
    xt, yt = t
    xq, yq = q
    xp, yp = p
    if xt != xq:
        lam = f12_mul(f12_sub(yq, yt), f12_inv(f12_sub(xq, xt)))
        return f12_sub(f12_sub(yp, yt), f12_mul(lam, f12_sub(xp, xt)))
    if yt == yq:
        lam = f12_mul(f12_scale(f12_mul(xt, xt), 3), f12_inv(f12_scale(yt, 2)))
        return f12_sub(f12_sub(yp, yt), f12_mul(lam, f12_sub(xp, xt)))
    # vertical line
    return f12_sub(xp, xt)


def _frobenius_point(pt):
    return (f12_pow(pt[0], P), f12_pow(pt[1], P))


def miller_loop(p_g1, q_g2):
    """Miller value f_{6u+2,Q}(P) times the two Frobenius correction lines."""
    if p_g1 is None or q_g2 is None:
        return f12_one()
    p = embed_g1(p_g1)
    q = untwist(q_g2)
    t = q
    f = f12_one()
    for bit in bin(ATE_LOOP)[3:]:
        f = f12_mul(f12_sqr(f), _line(t, t, p))
        t = ec_double(FQ12, t)
        if bit == "1":
            f = f12_mul(f, _line(t, q, p))
            t = ec_add(FQ12, t, q)
    q1 = _frobenius_point(q)
    q2 = ec_neg(FQ12, _frobenius_point(q1))
    f = f12_mul(f, _line(t, q1, p))
    t = ec_add(FQ12, t, q1)
    f = f12_mul(f, _line(t, q2, p))
    return f


def final_exponentiation(f):
    return f12_pow(f, FINAL_EXP)


def pairing(p_g1, q_g2):
    return final_exponentiation(miller_loop(p_g1, q_g2))


def pairing_product_is_one(pairs):
    """True iff prod_k e(P_k, Q_k) == 1, with one shared final exponentiation."""
    f = f12_one()
    for p_g1, q_g2 in pairs:
        f = f12_mul(f, miller_loop(p_g1, q_g2))
    return f12_is_one(final_exponentiation(f))
