"""BN254 fields and curve groups, written out plainly for the CPU oracle.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct CPU
statement of what the GPU prover computes.  Only the test suite, the smoke
check and the CPU-baseline leg of the benchmark may import it; the product
library never does.

The paper proves matrix products with Groth16 over a pairing-friendly curve
but does not name the curve (Section IV, implementation details: the backend
is libsnark's Groth16).  This oracle fixes BN254, the Barreto-Naehrig curve
with parameter u below; every constant is derived here from u rather than
typed in, so a reader can check them against the BN family's defining
polynomials.

Representation (chosen for readability, not speed):
  * Fq, Fr elements are Python ints in [0, modulus).
  * Fq2 = Fq[i]/(i^2 + 1) elements are tuples (c0, c1) meaning c0 + c1*i.
  * Fq12 elements are lists of 12 Fq ints: coefficients of a polynomial in w
    modulo w^12 - 18 w^6 + 82.  With w^6 = xi = 9 + i this is the usual
    sextic extension of Fq2 (i = w^6 - 9 gives i^2 = -1).
  * Affine points are tuples (x, y); the point at infinity is None.
"""

# --------------------------------------------------------------------------
# Parameters (BN family: p(u) = 36u^4+36u^3+24u^2+6u+1,
#                        r(u) = 36u^4+36u^3+18u^2+6u+1, trace t = 6u^2+1)
# --------------------------------------------------------------------------
U = 4965661367192848881
P = 36 * U**4 + 36 * U**3 + 24 * U**2 + 6 * U + 1
R = 36 * U**4 + 36 * U**3 + 18 * U**2 + 6 * U + 1
TRACE = 6 * U**2 + 1
B_G1 = 3  # E: y^2 = x^3 + 3 over Fq

G1_GEN = (1, 2)

# Standard BN254 G2 generator on the D-type twist E': y^2 = x^3 + 3/(9+i).
G2_GEN = (
    (10857046999023057135944570762232829481370756359578518086990519993285655852781,
     11559732032986387107991004021392285783925812861821192530917403151452391805634),
    (8495653923123431417604973247489272438418190587263600148770280649306958101930,
     4082367875863433681332203403145435568316851327593401208105741076214120093531),
)


# --------------------------------------------------------------------------
# Prime fields
# --------------------------------------------------------------------------
def fq_inv(a):
    if a % P == 0:
        raise ZeroDivisionError("inverse of zero in Fq")
    return pow(a, -1, P)


def fr_inv(a):
    if a % R == 0:
        raise ZeroDivisionError("inverse of zero in Fr")
    return pow(a, -1, R)


def fq_sqrt(a):
    """Square root in Fq (p = 3 mod 4); None if a is a non-residue."""
    a %= P
    s = pow(a, (P + 1) // 4, P)
    return s if s * s % P == a else None


# --------------------------------------------------------------------------
# Fq2 = Fq[i]/(i^2+1)
# --------------------------------------------------------------------------
F2_ZERO = (0, 0)
F2_ONE = (1, 0)
XI = (9, 1)  # the sextic non-residue 9 + i


def f2(a):
    return (a[0] % P, a[1] % P)


def f2_add(a, b):
    return ((a[0] + b[0]) % P, (a[1] + b[1]) % P)


def f2_sub(a, b):
    return ((a[0] - b[0]) % P, (a[1] - b[1]) % P)


def f2_neg(a):
    return ((-a[0]) % P, (-a[1]) % P)


def f2_mul(a, b):
    # (a0 + a1 i)(b0 + b1 i) = (a0 b0 - a1 b1) + (a0 b1 + a1 b0) i
    return ((a[0] * b[0] - a[1] * b[1]) % P, (a[0] * b[1] + a[1] * b[0]) % P)


def f2_scale(a, k):
    return (a[0] * k % P, a[1] * k % P)


def f2_sqr(a):
    return f2_mul(a, a)


def f2_inv(a):
    # 1/(a0 + a1 i) = (a0 - a1 i)/(a0^2 + a1^2)
    d = fq_inv(a[0] * a[0] + a[1] * a[1])
    return (a[0] * d % P, (-a[1]) * d % P)


def f2_conj(a):
    return (a[0], (-a[1]) % P)


def f2_pow(a, e):
    out = F2_ONE
    base = a
    while e:
        if e & 1:
            out = f2_mul(out, base)
        base = f2_sqr(base)
        e >>= 1
    return out


def f2_is_zero(a):
    return a[0] % P == 0 and a[1] % P == 0


B_G2 = f2_mul((3, 0), f2_inv(XI))  # twist coefficient 3/(9+i)


# --------------------------------------------------------------------------
# Fq12 = Fq[w]/(w^12 - 18 w^6 + 82)
# --------------------------------------------------------------------------
F12_DEG = 12


def f12_one():
    return [1] + [0] * 11


def f12_zero():
    return [0] * 12


def f12_from_fq(a):
    return [a % P] + [0] * 11


def f12_from_f2(a):
    # a0 + a1 i with i = w^6 - 9
    out = [0] * 12
    out[0] = (a[0] - 9 * a[1]) % P
    out[6] = a[1] % P
    return out


def f12_add(a, b):
    return [(x + y) % P for x, y in zip(a, b)]


def f12_sub(a, b):
    return [(x - y) % P for x, y in zip(a, b)]


def f12_neg(a):
    return [(-x) % P for x in a]


def f12_scale(a, k):
    return [x * k % P for x in a]


def f12_mul(a, b):
    prod = [0] * 23
    for i, x in enumerate(a):
        if x:
            for j, y in enumerate(b):
                prod[i + j] += x * y
    # reduce with w^12 = 18 w^6 - 82, from the top down
    for d in range(22, 11, -1):
        c = prod[d]
        if c:
            prod[d] = 0
            prod[d - 6] += 18 * c
            prod[d - 12] -= 82 * c
    return [c % P for c in prod[:12]]


def f12_sqr(a):
    return f12_mul(a, a)


def f12_eq(a, b):
    return all((x - y) % P == 0 for x, y in zip(a, b))


def f12_is_one(a):
    return f12_eq(a, f12_one())


def f12_pow(a, e):
    out = f12_one()
    base = a
    while e:
        if e & 1:
            out = f12_mul(out, base)
        base = f12_sqr(base)
        e >>= 1
    return out


def _poly_divmod(num, den):
    """Polynomial division over Fq; lists are low-degree first, den monic-izable."""
    num = list(num)
    while num and num[-1] % P == 0:
        num.pop()
    dd = len(den) - 1
    while dd >= 0 and den[dd] % P == 0:
        dd -= 1
    inv_lead = fq_inv(den[dd])
    q = [0] * max(len(num) - dd, 1)
    while len(num) - 1 >= dd and num:
        shift = len(num) - 1 - dd
        c = num[-1] * inv_lead % P
        q[shift] = c
        for k in range(dd + 1):
            num[shift + k] = (num[shift + k] - c * den[k]) % P
        while num and num[-1] % P == 0:
            num.pop()
    return q, num


def f12_inv(a):
    """Inverse via the extended Euclidean algorithm on polynomials over Fq."""
    modulus = [82, 0, 0, 0, 0, 0, (-18) % P, 0, 0, 0, 0, 0, 1]
    r0, r1 = modulus, [x % P for x in a]
    s0, s1 = [0], [1]
    while any(x % P for x in r1):
        q, rem = _poly_divmod(r0, r1)
        # s_new = s0 - q*s1
        qs = [0] * (len(q) + len(s1))
        for i, x in enumerate(q):
            for j, y in enumerate(s1):
                qs[i + j] += x * y
        n = max(len(s0), len(qs))
        s_new = [((s0[k] if k < len(s0) else 0) - (qs[k] if k < len(qs) else 0)) % P for k in range(n)]
        r0, r1 = r1, rem if rem else [0]
        s0, s1 = s1, s_new
    # r0 is a nonzero constant (gcd); scale
    while len(r0) > 1 and r0[-1] % P == 0:
        r0.pop()
    if len(r0) != 1 or r0[0] % P == 0:
        raise ZeroDivisionError("element not invertible in Fq12")
    c = fq_inv(r0[0])
    out = [0] * 12
    # reduce s0 modulo the modulus polynomial
    _, s_red = _poly_divmod(s0, modulus)
    for k, x in enumerate(s_red):
        out[k] = x * c % P
    return out


# --------------------------------------------------------------------------
# Generic short-Weierstrass affine arithmetic (y^2 = x^3 + b), a = 0.
# `ops` bundles the coordinate field's operations so one copy of the group
# law serves G1 (over Fq), G2 (over Fq2) and the pairing's E(Fq12).
# --------------------------------------------------------------------------
class _Field:
    def __init__(self, add, sub, mul, inv, neg, zero, one, eq, from_int):
        self.add, self.sub, self.mul, self.inv, self.neg = add, sub, mul, inv, neg
        self.zero, self.one, self.eq, self.from_int = zero, one, eq, from_int


FQ = _Field(lambda a, b: (a + b) % P, lambda a, b: (a - b) % P, lambda a, b: a * b % P,
            fq_inv, lambda a: (-a) % P, 0, 1, lambda a, b: (a - b) % P == 0, lambda k: k % P)
FQ2 = _Field(f2_add, f2_sub, f2_mul, f2_inv, f2_neg, F2_ZERO, F2_ONE,
             lambda a, b: f2_is_zero(f2_sub(a, b)), lambda k: (k % P, 0))
FQ12 = _Field(f12_add, f12_sub, f12_mul, f12_inv, f12_neg, f12_zero(), f12_one(), f12_eq,
              f12_from_fq)


def ec_on_curve(F, pt, b):
    if pt is None:
        return True
    x, y = pt
    return F.eq(F.mul(y, y), F.add(F.mul(F.mul(x, x), x), b))


def ec_neg(F, pt):
    if pt is None:
        return None
    return (pt[0], F.neg(pt[1]))


def ec_double(F, pt):
    if pt is None:
        return None
    x, y = pt
    if F.eq(y, F.zero):
        return None
    # lambda = 3x^2 / 2y
    lam = F.mul(F.mul(F.from_int(3), F.mul(x, x)), F.inv(F.mul(F.from_int(2), y)))
    x3 = F.sub(F.mul(lam, lam), F.mul(F.from_int(2), x))
    y3 = F.sub(F.mul(lam, F.sub(x, x3)), y)
    return (x3, y3)


def ec_add(F, p1, p2):
    if p1 is None:
        return p2
    if p2 is None:
        return p1
    x1, y1 = p1
    x2, y2 = p2
    if F.eq(x1, x2):
        if F.eq(y1, y2):
            return ec_double(F, p1)
        return None
    lam = F.mul(F.sub(y2, y1), F.inv(F.sub(x2, x1)))
    x3 = F.sub(F.sub(F.mul(lam, lam), x1), x2)
    y3 = F.sub(F.mul(lam, F.sub(x1, x3)), y1)
    return (x3, y3)


def ec_mul(F, pt, k):
    """Double-and-add scalar multiplication, k >= 0 any size."""
    if k < 0:
        return ec_mul(F, ec_neg(F, pt), -k)
    acc = None
    base = pt
    while k:
        if k & 1:
            acc = ec_add(F, acc, base)
        base = ec_double(F, base)
        k >>= 1
    return acc


def ec_eq(F, p1, p2):
    if p1 is None or p2 is None:
        return p1 is None and p2 is None
    return F.eq(p1[0], p2[0]) and F.eq(p1[1], p2[1])


# --------------------------------------------------------------------------
# G1 over Fq.  Jacobian coordinates are used for the bulk scalar
# multiplications (setup and MSM) only to avoid one inversion per addition;
# results are always returned affine.
# --------------------------------------------------------------------------
def g1_on_curve(pt):
    return ec_on_curve(FQ, pt, B_G1)


def g1_add(a, b):
    return ec_add(FQ, a, b)


def g1_neg(a):
    return ec_neg(FQ, a)


def g1_eq(a, b):
    return ec_eq(FQ, a, b)


def _jac_double(X, Y, Z):
    # a = 0 doubling: S = 4XY^2, M = 3X^2, X' = M^2 - 2S, Y' = M(S - X') - 8Y^4, Z' = 2YZ
    if Z == 0 or Y == 0:
        return (1, 1, 0)
    YY = Y * Y % P
    S = 4 * X * YY % P
    M = 3 * X * X % P
    X3 = (M * M - 2 * S) % P
    Y3 = (M * (S - X3) - 8 * YY * YY) % P
    Z3 = 2 * Y * Z % P
    return (X3, Y3, Z3)


def _jac_add(p1, p2):
    X1, Y1, Z1 = p1
    X2, Y2, Z2 = p2
    if Z1 == 0:
        return p2
    if Z2 == 0:
        return p1
    Z1Z1 = Z1 * Z1 % P
    Z2Z2 = Z2 * Z2 % P
    U1 = X1 * Z2Z2 % P
    U2 = X2 * Z1Z1 % P
    S1 = Y1 * Z2 * Z2Z2 % P
    S2 = Y2 * Z1 * Z1Z1 % P
    if U1 == U2:
        if S1 == S2:
            return _jac_double(X1, Y1, Z1)
        return (1, 1, 0)
    H = (U2 - U1) % P
    Rr = (S2 - S1) % P
    HH = H * H % P
    HHH = H * HH % P
    V = U1 * HH % P
    X3 = (Rr * Rr - HHH - 2 * V) % P
    Y3 = (Rr * (V - X3) - S1 * HHH) % P
    Z3 = Z1 * Z2 * H % P
    return (X3, Y3, Z3)


def _jac_to_affine(p):
    X, Y, Z = p
    if Z % P == 0:
        return None
    zi = fq_inv(Z)
    zi2 = zi * zi % P
    return (X * zi2 % P, Y * zi2 * zi % P)


def _jac_from_affine(a):
    if a is None:
        return (1, 1, 0)
    return (a[0], a[1], 1)


def g1_mul(pt, k):
    """[k]pt by double-and-add (k reduced mod r: pt is assumed of order r)."""
    k %= R
    acc = (1, 1, 0)
    base = _jac_from_affine(pt)
    while k:
        if k & 1:
            acc = _jac_add(acc, base)
        base = _jac_double(*base)
        k >>= 1
    return _jac_to_affine(acc)


def g1_mul_any(pt, k):
    """[k]pt by double-and-add without reducing k (for order checks)."""
    acc = (1, 1, 0)
    base = _jac_from_affine(pt)
    while k:
        if k & 1:
            acc = _jac_add(acc, base)
        base = _jac_double(*base)
        k >>= 1
    return _jac_to_affine(acc)


def g1_msm(points, scalars):
    """Sum_i [s_i] P_i, one double-and-add per term, summed in Jacobian form."""
    acc = (1, 1, 0)
    for pt, s in zip(points, scalars):
        k = s % R
        if pt is None or k == 0:
            continue
        term = (1, 1, 0)
        base = _jac_from_affine(pt)
        while k:
            if k & 1:
                term = _jac_add(term, base)
            base = _jac_double(*base)
            k >>= 1
        acc = _jac_add(acc, term)
    return _jac_to_affine(acc)


# --------------------------------------------------------------------------
# G2 over Fq2 (affine arithmetic; the oracle's G2 work is small)
# --------------------------------------------------------------------------
def g2_on_curve(pt):
    return ec_on_curve(FQ2, pt, B_G2)


def g2_add(a, b):
    return ec_add(FQ2, a, b)


def g2_neg(a):
    return ec_neg(FQ2, a)


def g2_eq(a, b):
    return ec_eq(FQ2, a, b)


def _j2_double(p):
    X, Y, Z = p
    if f2_is_zero(Z) or f2_is_zero(Y):
        return (F2_ONE, F2_ONE, F2_ZERO)
    YY = f2_sqr(Y)
    S = f2_scale(f2_mul(X, YY), 4)
    M = f2_scale(f2_sqr(X), 3)
    X3 = f2_sub(f2_sqr(M), f2_scale(S, 2))
    Y3 = f2_sub(f2_mul(M, f2_sub(S, X3)), f2_scale(f2_sqr(YY), 8))
    Z3 = f2_scale(f2_mul(Y, Z), 2)
    return (X3, Y3, Z3)


def _j2_add(p1, p2):
    X1, Y1, Z1 = p1
    X2, Y2, Z2 = p2
    if f2_is_zero(Z1):
        return p2
    if f2_is_zero(Z2):
        return p1
    Z1Z1 = f2_sqr(Z1)
    Z2Z2 = f2_sqr(Z2)
    U1 = f2_mul(X1, Z2Z2)
    U2 = f2_mul(X2, Z1Z1)
    S1 = f2_mul(f2_mul(Y1, Z2), Z2Z2)
    S2 = f2_mul(f2_mul(Y2, Z1), Z1Z1)
    if f2_is_zero(f2_sub(U1, U2)):
        if f2_is_zero(f2_sub(S1, S2)):
            return _j2_double(p1)
        return (F2_ONE, F2_ONE, F2_ZERO)
    H = f2_sub(U2, U1)
    Rr = f2_sub(S2, S1)
    HH = f2_sqr(H)
    HHH = f2_mul(H, HH)
    V = f2_mul(U1, HH)
    X3 = f2_sub(f2_sub(f2_sqr(Rr), HHH), f2_scale(V, 2))
    Y3 = f2_sub(f2_mul(Rr, f2_sub(V, X3)), f2_mul(S1, HHH))
    Z3 = f2_mul(f2_mul(Z1, Z2), H)
    return (X3, Y3, Z3)


def _j2_to_affine(p):
    X, Y, Z = p
    if f2_is_zero(Z):
        return None
    zi = f2_inv(Z)
    zi2 = f2_sqr(zi)
    return (f2_mul(X, zi2), f2_mul(f2_mul(Y, zi2), zi))


def _j2_from_affine(a):
    if a is None:
        return (F2_ONE, F2_ONE, F2_ZERO)
    return (a[0], a[1], F2_ONE)


def g2_mul_any(pt, k):
    acc = (F2_ONE, F2_ONE, F2_ZERO)
    base = _j2_from_affine(pt)
    while k:
        if k & 1:
            acc = _j2_add(acc, base)
        base = _j2_double(base)
        k >>= 1
    return _j2_to_affine(acc)


def g2_mul(pt, k):
    """[k]pt for pt in the order-r subgroup (k reduced mod r)."""
    return g2_mul_any(pt, k % R)


def g2_msm(points, scalars):
    acc = (F2_ONE, F2_ONE, F2_ZERO)
    for pt, s in zip(points, scalars):
        k = s % R
        if pt is None or k == 0:
            continue
        term = (F2_ONE, F2_ONE, F2_ZERO)
        base = _j2_from_affine(pt)
        while k:
            if k & 1:
                term = _j2_add(term, base)
            base = _j2_double(base)
            k >>= 1
        acc = _j2_add(acc, term)
    return _j2_to_affine(acc)


def g2_in_subgroup(pt):
    return pt is not None and g2_on_curve(pt) and g2_mul_any(pt, R) is None


def g1_valid(pt):
    """On the curve and not infinity (G1 has cofactor 1)."""
    return pt is not None and g1_on_curve(pt)
