"""Pins for the oracle's BN254 fields, groups and pairing (no GPU).

Each test checks the oracle against something other than itself: the BN
family's closed forms, primality, group orders, brute-force repeated
addition, and the defining properties of a pairing.
"""
import random

import pytest

from oracle import bn254 as bn
from oracle import pairing as pr


def _is_probable_prime(n, rounds=32, seed=1):
    if n < 2:
        return False
    for p in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    rng = random.Random(seed)
    for _ in range(rounds):
        a = rng.randrange(2, n - 1)
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def test_bn_parameters_closed_forms():
    u = bn.U
    assert bn.P == 36 * u**4 + 36 * u**3 + 24 * u**2 + 6 * u + 1
    assert bn.R == 36 * u**4 + 36 * u**3 + 18 * u**2 + 6 * u + 1
    # Hasse: #E(Fq) = p + 1 - t with t = 6u^2 + 1 equals r (cofactor 1)
    assert bn.P + 1 - (6 * u * u + 1) == bn.R
    assert bn.P.bit_length() == 254 and bn.R.bit_length() == 254
    assert bn.P % 4 == 3
    # well-known hex forms of the BN254 moduli
    assert hex(bn.P) == "0x30644e72e131a029b85045b68181585d97816a916871ca8d3c208c16d87cfd47"
    assert hex(bn.R) == "0x30644e72e131a029b85045b68181585d2833e84879b9709143e1f593f0000001"


def test_moduli_are_prime():
    assert _is_probable_prime(bn.P)
    assert _is_probable_prime(bn.R)


def test_two_adicity_and_generator():
    r1 = bn.R - 1
    k = 0
    while r1 % 2 == 0:
        r1 //= 2
        k += 1
    assert k == 28
    # 5 is a quadratic non-residue mod r, so 5^((r-1)/2^28) has order exactly 2^28
    assert pow(5, (bn.R - 1) // 2, bn.R) == bn.R - 1


def test_g1_generator_order():
    assert bn.g1_on_curve(bn.G1_GEN)
    assert bn.g1_mul_any(bn.G1_GEN, bn.R) is None
    assert bn.g1_mul_any(bn.G1_GEN, bn.R - 1) == bn.g1_neg(bn.G1_GEN)


def test_g2_generator_order_and_twist_cofactor():
    assert bn.g2_on_curve(bn.G2_GEN)
    assert bn.g2_mul_any(bn.G2_GEN, bn.R) is None
    # a random point on the twist: its order divides r (2p - r) but usually not r
    rng = random.Random(7)
    while True:
        x = (rng.randrange(bn.P), rng.randrange(bn.P))
        rhs = bn.f2_add(bn.f2_mul(bn.f2_sqr(x), x), bn.B_G2)
        # square root in Fq2 via norm: try the (p^2+7)/16-free route by brute check
        y = _f2_sqrt(rhs)
        if y is not None:
            break
    q = (x, y)
    assert bn.g2_on_curve(q)
    assert bn.g2_mul_any(q, bn.R * (2 * bn.P - bn.R)) is None
    assert bn.g2_mul_any(q, bn.R) is not None


def _f2_sqrt(a):
    # Fq2 square root for p = 3 mod 4 (a standard complex-method formula)
    a0, a1 = a
    if a1 == 0:
        s = bn.fq_sqrt(a0)
        if s is not None:
            return (s, 0)
        s = bn.fq_sqrt((-a0) % bn.P)
        return (0, s) if s is not None else None
    norm = (a0 * a0 + a1 * a1) % bn.P
    n = bn.fq_sqrt(norm)
    if n is None:
        return None
    for cand in ((a0 + n) * pow(2, -1, bn.P) % bn.P, (a0 - n) * pow(2, -1, bn.P) % bn.P):
        x0 = bn.fq_sqrt(cand)
        if x0 is not None and x0 != 0:
            x1 = a1 * pow(2 * x0, -1, bn.P) % bn.P
            y = (x0, x1)
            if bn.f2_sqr(y) == (a0 % bn.P, a1 % bn.P):
                return y
    return None


def test_fq2_arithmetic_against_definition():
    rng = random.Random(3)
    for _ in range(20):
        a = (rng.randrange(bn.P), rng.randrange(bn.P))
        b = (rng.randrange(bn.P), rng.randrange(bn.P))
        # (a0 + a1 i)(b0 + b1 i) with i^2 = -1 expanded by hand
        assert bn.f2_mul(a, b) == ((a[0] * b[0] - a[1] * b[1]) % bn.P, (a[0] * b[1] + a[1] * b[0]) % bn.P)
        assert bn.f2_mul(a, bn.f2_inv(a)) == (1, 0)
    assert bn.f2_sqr((0, 1)) == (bn.P - 1, 0)


def test_fq12_tower_relations():
    i12 = bn.f12_from_f2((0, 1))
    assert bn.f12_eq(bn.f12_sqr(i12), bn.f12_neg(bn.f12_one()))
    w = [0, 1] + [0] * 10
    w6 = bn.f12_pow(w, 6)
    assert bn.f12_eq(w6, bn.f12_from_f2(bn.XI))
    rng = random.Random(5)
    a = [rng.randrange(bn.P) for _ in range(12)]
    assert bn.f12_is_one(bn.f12_mul(a, bn.f12_inv(a)))
    # Fq2 embeds multiplicatively
    x = (rng.randrange(bn.P), rng.randrange(bn.P))
    y = (rng.randrange(bn.P), rng.randrange(bn.P))
    assert bn.f12_eq(bn.f12_mul(bn.f12_from_f2(x), bn.f12_from_f2(y)), bn.f12_from_f2(bn.f2_mul(x, y)))


def test_scalar_mul_matches_repeated_addition():
    acc1, acc2 = None, None
    for k in range(1, 40):
        acc1 = bn.g1_add(acc1, bn.G1_GEN)
        acc2 = bn.g2_add(acc2, bn.G2_GEN)
        assert bn.g1_eq(bn.g1_mul(bn.G1_GEN, k), acc1)
        assert bn.g2_eq(bn.g2_mul(bn.G2_GEN, k), acc2)


def test_msm_brute_force_and_edges():
    rng = random.Random(11)
    for n in range(0, 9):
        pts = [bn.g1_mul(bn.G1_GEN, rng.randrange(1, 1 << 20)) for _ in range(n)]
        sc = [rng.randrange(0, 1 << 10) for _ in range(n)]
        want = None
        for p, s in zip(pts, sc):
            for _ in range(s):
                want = bn.g1_add(want, p)
        assert bn.g1_eq(bn.g1_msm(pts, sc), want)
    g = bn.G1_GEN
    assert bn.g1_msm([], []) is None
    assert bn.g1_msm([g], [0]) is None
    assert bn.g1_msm([g], [bn.R - 1]) == bn.g1_neg(g)
    assert bn.g1_msm([g, bn.g1_neg(g)], [5, 5]) is None
    assert bn.g1_eq(bn.g1_msm([g, g, g], [1, 2, 3]), bn.g1_mul(g, 6))
    assert bn.g1_eq(bn.g1_msm([None, g], [9, 2]), bn.g1_mul(g, 2))
    # discrete-log identity: bases [k_i]G give [sum s_i k_i]G
    ks = [rng.randrange(bn.R) for _ in range(6)]
    ss = [rng.randrange(bn.R) for _ in range(6)]
    pts = [bn.g1_mul(g, k) for k in ks]
    assert bn.g1_eq(bn.g1_msm(pts, ss), bn.g1_mul(g, sum(a * b for a, b in zip(ks, ss))))
    q = bn.G2_GEN
    pts2 = [bn.g2_mul(q, k) for k in ks[:3]]
    assert bn.g2_eq(bn.g2_msm(pts2, ss[:3]), bn.g2_mul(q, sum(a * b for a, b in zip(ks[:3], ss[:3]))))


@pytest.mark.slow
def test_pairing_bilinear_nondegenerate_order_r():
    rng = random.Random(13)
    e = pr.pairing(bn.G1_GEN, bn.G2_GEN)
    assert not bn.f12_is_one(e)
    assert bn.f12_is_one(bn.f12_pow(e, bn.R))
    a, b = rng.randrange(1, bn.R), rng.randrange(1, bn.R)
    lhs = pr.pairing(bn.g1_mul(bn.G1_GEN, a), bn.g2_mul(bn.G2_GEN, b))
    assert bn.f12_eq(lhs, bn.f12_pow(e, a * b % bn.R))
    # additivity in each argument
    p1, p2 = bn.g1_mul(bn.G1_GEN, 3), bn.g1_mul(bn.G1_GEN, 5)
    assert bn.f12_eq(pr.pairing(bn.g1_add(p1, p2), bn.G2_GEN),
                     bn.f12_mul(pr.pairing(p1, bn.G2_GEN), pr.pairing(p2, bn.G2_GEN)))
    q1, q2 = bn.g2_mul(bn.G2_GEN, 7), bn.g2_mul(bn.G2_GEN, 11)
    assert bn.f12_eq(pr.pairing(bn.G1_GEN, bn.g2_add(q1, q2)),
                     bn.f12_mul(pr.pairing(bn.G1_GEN, q1), pr.pairing(bn.G1_GEN, q2)))
    assert pr.pairing_product_is_one([(bn.g1_mul(bn.G1_GEN, a), bn.G2_GEN),
                                      (bn.g1_neg(bn.G1_GEN), bn.g2_mul(bn.G2_GEN, a))])
