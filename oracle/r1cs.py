"""Constraint systems for Y = X W, written out row by row for the CPU oracle.

TEST INFRASTRUCTURE ONLY (see oracle/bn254.py).

Two constraint systems are built for X in Z^{a x n}, W in Z^{n x b}:

PLAIN (Section III-A, the "vanilla" circuit: one constraint per product).
    For each output y_ij and each k < n there is one multiplication
    constraint  x_ik * w_kj = C.  For k < n-1 the right side is a fresh
    witness p_ijk holding the product; for k = n-1 the right side is
    y_ij - sum_{k'<n-1} p_ijk', which folds the output sum into the last
    product's constraint.  That gives exactly a*b*n constraints.

CRPC_PSQ (Section III-A, the generalised CRPC identity, combined with the
prefix-sum query of Section III-B).  With a public field element z in place
of the formal variable Z,
    X_k(z) = sum_i z^(i b) x_ik,   W_k(z) = sum_j z^j w_kj,
    Y(z)   = sum_{i,j} z^(i b + j) y_ij,
and the witness holds prefix sums s_k = sum_{k'<=k} X_k'(z) W_k'(z) instead of
the products (Section III-B stores a_7, a_8, a_9 as running sums).  Row k is
    X_k(z) * W_k(z) = s_k - s_{k-1}            (k < n-1, s_{-1} = 0)
    X_k(z) * W_k(z) = Y(z) - s_{n-2}           (k = n-1),
so n constraints in all and the last prefix sum is never stored: it is Y(z).

Three further systems reproduce the other rows of the paper's ablation
(Table II) with the same variables and inputs:
  PLAIN_ADD  the literal vanilla circuit of Section III-B: n product
             constraints x_ik w_kj = p_ijk per output, then one long-addition
             constraint (sum_k p_ijk) * 1 = y_ij, so a*b*(n+1) constraints and
             the products appear as left wires;
  PLAIN_PSQ  the per-product circuit holding prefix sums s_ijk instead of
             products (Section III-B applied without CRPC), a*b*n constraints;
  CRPC       CRPC without prefix sums: n product constraints
             X_k(z) W_k(z) = P_k and one addition (sum_k P_k) * 1 = Y(z).

Variable order (shared with the GPU library's proving key layout):
    0                      the constant 1
    1 + i n + k            x_ik         (public)
    1 + a n + i b + j      y_ij         (public)
    1 + l + k b + j        w_kj         (witness), l = a n + a b
    1 + l + n b + t        auxiliary t  (witness):
                             PLAIN, PLAIN_PSQ  t = (i b + j)(n-1) + k, k < n-1
                             PLAIN_ADD         t = (i b + j) n + k
                             CRPC_PSQ          t = k < n-1 (prefix sums)
                             CRPC              t = k < n   (products)
After the m multiplication rows come l + 1 input-consistency rows: row m + t
has A = variable t, B = C = 0, which makes the public-input polynomials
linearly independent.  Rows from m + l + 1 up to the domain size N are zero.
"""
from collections import namedtuple

from .bn254 import R

PLAIN = 0
CRPC_PSQ = 1
PLAIN_ADD = 2
PLAIN_PSQ = 3
CRPC = 4
KIND_NAMES = {PLAIN: "plain", CRPC_PSQ: "crpc_psq", PLAIN_ADD: "plain_add", PLAIN_PSQ: "plain_psq",
              CRPC: "crpc"}
CRPC_KINDS = (CRPC_PSQ, CRPC)

Shape = namedtuple("Shape", "a n b")


def num_public(s):
    return s.a * s.n + s.a * s.b


def num_aux(s, kind):
    if kind in (PLAIN, PLAIN_PSQ):
        return s.a * s.b * (s.n - 1)
    if kind == PLAIN_ADD:
        return s.a * s.b * s.n
    if kind == CRPC_PSQ:
        return s.n - 1
    if kind == CRPC:
        return s.n
    raise ValueError("unknown kind")


def num_constraints(s, kind):
    if kind in (PLAIN, PLAIN_PSQ):
        return s.a * s.b * s.n
    if kind == PLAIN_ADD:
        return s.a * s.b * (s.n + 1)
    if kind == CRPC_PSQ:
        return s.n
    if kind == CRPC:
        return s.n + 1
    raise ValueError("unknown kind")


def num_vars(s, kind):
    return 1 + num_public(s) + s.n * s.b + num_aux(s, kind)


def domain_size(s, kind):
    rows = num_constraints(s, kind) + num_public(s) + 1
    n = 1
    while n < rows:
        n <<= 1
    return n


def var_x(s, i, k):
    return 1 + i * s.n + k


def var_y(s, i, j):
    return 1 + s.a * s.n + i * s.b + j


def var_w(s, k, j):
    return 1 + num_public(s) + k * s.b + j


def var_aux(s, t):
    return 1 + num_public(s) + s.n * s.b + t


def first_witness(s):
    """Index of the first witness variable; 0..l are the constant and public inputs."""
    return 1 + num_public(s)


def z_powers(s, z):
    """[z^e for e < a*b]: the weights of the CRPC polynomials (Section III-A)."""
    if z is None or z % R == 0:
        raise ValueError("the CRPC kinds need a nonzero public z")
    return [pow(z, e, R) for e in range(s.a * s.b)]


def row(s, kind, c, zp=None):
    """(A, B, C) of row c as {variable: coefficient} dicts (rows past the last are empty).

    zp: z_powers(s, z) for the CRPC kinds.
    """
    m = num_constraints(s, kind)
    ell = num_public(s)
    if c >= m:
        t = c - m
        return ({t: 1}, {}, {}) if t <= ell else ({}, {}, {})
    if kind in (PLAIN, PLAIN_PSQ):
        ij, k = divmod(c, s.n)
        i, j = divmod(ij, s.b)
        base = ij * (s.n - 1)
        A = {var_x(s, i, k): 1}
        B = {var_w(s, k, j): 1}
        if kind == PLAIN:
            if k < s.n - 1:
                C = {var_aux(s, base + k): 1}
            else:
                C = {var_y(s, i, j): 1}
                for kk in range(s.n - 1):
                    C[var_aux(s, base + kk)] = R - 1
        else:
            C = {var_aux(s, base + k): 1} if k < s.n - 1 else {var_y(s, i, j): 1}
            if k >= 1:
                C[var_aux(s, base + k - 1)] = R - 1
        return A, B, C
    if kind == PLAIN_ADD:
        ij, k = divmod(c, s.n + 1)
        i, j = divmod(ij, s.b)
        base = ij * s.n
        if k < s.n:
            return {var_x(s, i, k): 1}, {var_w(s, k, j): 1}, {var_aux(s, base + k): 1}
        return {var_aux(s, base + kk): 1 for kk in range(s.n)}, {0: 1}, {var_y(s, i, j): 1}
    if kind == CRPC_PSQ:
        k = c
        A = {var_x(s, i, k): zp[i * s.b] for i in range(s.a)}
        B = {var_w(s, k, j): zp[j] for j in range(s.b)}
        if k < s.n - 1:
            C = {var_aux(s, k): 1}
            if k >= 1:
                C[var_aux(s, k - 1)] = R - 1
        else:
            C = {var_y(s, i, j): zp[i * s.b + j] for i in range(s.a) for j in range(s.b)}
            if s.n >= 2:
                C[var_aux(s, s.n - 2)] = R - 1
        return A, B, C
    if kind == CRPC:
        if c < s.n:
            k = c
            return ({var_x(s, i, k): zp[i * s.b] for i in range(s.a)},
                    {var_w(s, k, j): zp[j] for j in range(s.b)},
                    {var_aux(s, k): 1})
        return ({var_aux(s, k): 1 for k in range(s.n)}, {0: 1},
                {var_y(s, i, j): zp[i * s.b + j] for i in range(s.a) for j in range(s.b)})
    raise ValueError("unknown kind")


def rows(s, kind, z=None):
    """Yield (A, B, C) for every nonzero row in domain order.

    Rows 0..m-1 are the multiplication constraints, then come the l+1
    input-consistency rows (row m + t has A = variable t, B = C = 0).
    """
    if kind not in KIND_NAMES:
        raise ValueError("unknown kind")
    zp = z_powers(s, z) if kind in CRPC_KINDS else None
    for c in range(num_constraints(s, kind) + num_public(s) + 1):
        yield row(s, kind, c, zp)


def matmul(X, W):
    """Integer product of list-of-lists matrices."""
    a, n, b = len(X), len(W), len(W[0])
    return [[sum(X[i][k] * W[k][j] for k in range(n)) for j in range(b)] for i in range(a)]


def assignment(s, kind, X, W, z=None):
    """Full assignment (list of Fr ints) and the integer output Y = X W.

    Negative integers are encoded as r - |v| (their residue mod r).
    """
    Y = matmul(X, W)
    a = [1]
    a += [X[i][k] % R for i in range(s.a) for k in range(s.n)]
    a += [Y[i][j] % R for i in range(s.a) for j in range(s.b)]
    a += [W[k][j] % R for k in range(s.n) for j in range(s.b)]
    if kind == PLAIN:
        for i in range(s.a):
            for j in range(s.b):
                for k in range(s.n - 1):
                    a.append(X[i][k] * W[k][j] % R)
    elif kind == PLAIN_ADD:
        for i in range(s.a):
            for j in range(s.b):
                for k in range(s.n):
                    a.append(X[i][k] * W[k][j] % R)
    elif kind == PLAIN_PSQ:
        for i in range(s.a):
            for j in range(s.b):
                acc = 0
                for k in range(s.n - 1):
                    acc += X[i][k] * W[k][j]
                    a.append(acc % R)
    elif kind in CRPC_KINDS:
        acc = 0
        for k in range(s.n if kind == CRPC else s.n - 1):
            Xk = sum(pow(z, i * s.b, R) * X[i][k] for i in range(s.a)) % R
            Wk = sum(pow(z, j, R) * W[k][j] for j in range(s.b)) % R
            acc = (acc + Xk * Wk) % R
            a.append(Xk * Wk % R if kind == CRPC else acc)
    else:
        raise ValueError("unknown kind")
    assert len(a) == num_vars(s, kind)
    return a, Y


def dot(row, a):
    return sum(c * a[v] for v, c in row.items()) % R


def is_satisfied(s, kind, a, z=None):
    return all(dot(A, a) * dot(B, a) % R == dot(C, a) for A, B, C in rows(s, kind, z))


def eval_vectors(s, kind, a, z=None):
    """aev, bev, cev of length N: <A_c,a>, <B_c,a>, <C_c,a> at every domain row."""
    n_dom = domain_size(s, kind)
    aev, bev, cev = [], [], []
    for A, B, C in rows(s, kind, z):
        aev.append(dot(A, a))
        bev.append(dot(B, a))
        cev.append(dot(C, a))
    pad = n_dom - len(aev)
    return aev + [0] * pad, bev + [0] * pad, cev + [0] * pad


def left_wire_variables(s, kind, z=None):
    """Distinct variables with a nonzero coefficient in some multiplication row's A side.

    The paper counts these "left wires" (Section III-B); the consistency rows
    that follow the multiplication rows are not part of the circuit's count.
    """
    m = num_constraints(s, kind)
    seen = set()
    for c, (A, _, _) in enumerate(rows(s, kind, z)):
        if c >= m:
            break
        seen.update(v for v, coef in A.items() if coef % R)
    return seen
