"""Groth16 setup, prove and verify for the matmul circuits, for the CPU oracle.

TEST INFRASTRUCTURE ONLY (see oracle/bn254.py).

The paper's backend is Groth16 (Section II: Gen, Prove and Verify are the
three algorithms; Section IV: libsnark's Groth16 is the zkVC-G backend).  The
statement is Y = X W with X and Y public and W private (Section I, the client
sends X and receives Y with a proof).  The construction below is the standard
one from Groth's 2016 paper, written out with double-and-add scalar
multiplication and no precomputation:

  toxic waste (tau, alpha, beta, gamma, delta), public z for CRPC_PSQ

  pk:  [alpha]1 [beta]1 [beta]2 [delta]1 [delta]2
       A_i  = [u_i(tau)]1,  B1_i = [v_i(tau)]1,  B2_i = [v_i(tau)]2   (all i)
       L_i  = [(beta u_i + alpha v_i + w_i)(tau) / delta]1        (witness i)
       H_j  = [tau^j t(tau) / delta]1,  j = 0 .. N-2,  t(x) = x^N - 1
  vk:  [alpha]1 [beta]2 [gamma]2 [delta]2,
       IC_i = [(beta u_i + alpha v_i + w_i)(tau) / gamma]1        (i = 0 .. l)

  prove (r, s):
       A  = [alpha]1 + sum_i a_i A_i + r [delta]1
       B  = [beta]2  + sum_i a_i B2_i + s [delta]2
       B1 = [beta]1  + sum_i a_i B1_i + s [delta]1
       C  = sum_{witness i} a_i L_i + sum_j h_j H_j + s A + r B1 - r s [delta]1
  verify:
       e(A, B) = e([alpha]1, [beta]2) e(sum_{i<=l} a_i IC_i, [gamma]2) e(C, [delta]2)
       with A, C on E, B on the twist and in the order-r subgroup.

expected_proof_trapdoor computes the same proof from the toxic waste in
closed form (discrete logarithms of A, B, C), at O(N) field cost, so that
proofs at sizes too large for double-and-add can still be checked exactly.
"""
from collections import namedtuple

from .bn254 import (R, G1_GEN, G2_GEN, g1_mul, g2_mul, g1_add, g1_neg, g2_add, g1_msm, g2_msm,
                    g1_valid, g2_in_subgroup)
from .pairing import pairing_product_is_one
from . import qap
from . import r1cs

Toxic = namedtuple("Toxic", "tau alpha beta gamma delta")
Proof = namedtuple("Proof", "A B C")


def _inv(x):
    return pow(x, -1, R)


def setup(s, kind, toxic, z=None):
    """Honest key generation by double-and-add; practical only for small shapes."""
    n_dom = r1cs.domain_size(s, kind)
    u, v, w = qap.var_polys_at(s, kind, toxic.tau, z)
    ell = r1cs.num_public(s)
    nv = r1cs.num_vars(s, kind)
    d_inv = _inv(toxic.delta)
    g_inv = _inv(toxic.gamma)
    lin = [(toxic.beta * u[i] + toxic.alpha * v[i] + w[i]) % R for i in range(nv)]
    t_tau = (pow(toxic.tau, n_dom, R) - 1) % R
    pk = {
        "shape": s, "kind": kind, "N": n_dom, "z": z,
        "alpha1": g1_mul(G1_GEN, toxic.alpha),
        "beta1": g1_mul(G1_GEN, toxic.beta),
        "beta2": g2_mul(G2_GEN, toxic.beta),
        "delta1": g1_mul(G1_GEN, toxic.delta),
        "delta2": g2_mul(G2_GEN, toxic.delta),
        "A": [g1_mul(G1_GEN, x) for x in u],
        "B1": [g1_mul(G1_GEN, x) for x in v],
        "B2": [g2_mul(G2_GEN, x) for x in v],
        "L": [g1_mul(G1_GEN, lin[i] * d_inv) for i in range(ell + 1, nv)],
        "H": [g1_mul(G1_GEN, pow(toxic.tau, j, R) * t_tau % R * d_inv) for j in range(n_dom - 1)],
    }
    vk = {
        "shape": s, "kind": kind, "N": n_dom, "z": z,
        "alpha1": pk["alpha1"],
        "beta2": pk["beta2"],
        "gamma2": g2_mul(G2_GEN, toxic.gamma),
        "delta2": pk["delta2"],
        "IC": [g1_mul(G1_GEN, lin[i] * g_inv) for i in range(ell + 1)],
    }
    return pk, vk


def prove(pk, X, W, r, s_rand, quotient="coset"):
    """Honest prover: witness, quotient h, multi-scalar sums by double-and-add."""
    s, kind, z = pk["shape"], pk["kind"], pk["z"]
    a, Y = r1cs.assignment(s, kind, X, W, z)
    aev, bev, cev = r1cs.eval_vectors(s, kind, a, z)
    if quotient == "schoolbook":
        h = qap.quotient_schoolbook(aev, bev, cev)
    else:
        h = qap.quotient_coset(aev, bev, cev)
    ell = r1cs.num_public(s)
    A = g1_add(g1_add(pk["alpha1"], g1_msm(pk["A"], a)), g1_mul(pk["delta1"], r))
    B = g2_add(g2_add(pk["beta2"], g2_msm(pk["B2"], a)), g2_mul(pk["delta2"], s_rand))
    B1 = g1_add(g1_add(pk["beta1"], g1_msm(pk["B1"], a)), g1_mul(pk["delta1"], s_rand))
    C = g1_msm(pk["L"], a[ell + 1:])
    C = g1_add(C, g1_msm(pk["H"], h))
    C = g1_add(C, g1_mul(A, s_rand))
    C = g1_add(C, g1_mul(B1, r))
    C = g1_add(C, g1_neg(g1_mul(pk["delta1"], r * s_rand % R)))
    return Proof(A, B, C), Y


def public_inputs(s, X, Y):
    """a_0 .. a_l: the constant 1, then x row-major, then y row-major (mod r)."""
    out = [1]
    out += [X[i][k] % R for i in range(s.a) for k in range(s.n)]
    out += [Y[i][j] % R for i in range(s.a) for j in range(s.b)]
    return out


def verify(vk, X, Y, proof):
    """Groth16 verification equation plus on-curve and subgroup checks."""
    A, B, C = proof
    if not (g1_valid(A) and g1_valid(C) and g2_in_subgroup(B)):
        return False
    s = vk["shape"]
    if len(X) != s.a or len(Y) != s.a or any(len(row) != s.n for row in X) \
            or any(len(row) != s.b for row in Y):
        return False
    ic = g1_msm(vk["IC"], public_inputs(s, X, Y))
    return pairing_product_is_one([
        (A, B),
        (g1_neg(vk["alpha1"]), vk["beta2"]),
        (g1_neg(ic), vk["gamma2"]),
        (g1_neg(C), vk["delta2"]),
    ])


_SHARED = {}


def _row_sums(job):
    """Sums over rows c0 <= c < c1 of L_c(tau) <A_c,a>, ..., and of the witness-only parts."""
    s, kind, zp, tau, n_dom, c0, c1 = job
    a = _SHARED["a"]
    first = r1cs.first_witness(s)
    L = qap.lagrange_basis_range(n_dom, tau, c0, c1)
    sums = [0, 0, 0, 0, 0, 0]
    for c in range(c0, c1):
        lc = L[c - c0]
        for q, row in enumerate(r1cs.row(s, kind, c, zp)):
            full = wit = 0
            for v, coef in row.items():
                term = coef * a[v]
                full += term
                if v >= first:
                    wit += term
            sums[q] += lc * full
            sums[3 + q] += lc * wit
    return [x % R for x in sums]


def trapdoor_scalars(s, kind, toxic, X, W, r, s_rand, z=None, workers=1):
    """Discrete logarithms (base the generators) of every proof component.

    With L_c(tau) the Lagrange basis at tau:
      A(tau) = sum_c <A_c,a> L_c(tau), and likewise B(tau), C(tau);
      the witness-only parts use the assignment with a_0..a_l set to zero;
      h(tau) t(tau) = A(tau) B(tau) - C(tau) for a satisfying assignment.
    The row sums may be split over `workers` processes (same sums, any order).
    """
    n_dom = r1cs.domain_size(s, kind)
    a, Y = r1cs.assignment(s, kind, X, W, z)
    zp = r1cs.z_powers(s, z) if kind in r1cs.CRPC_KINDS else None
    nrows = r1cs.num_constraints(s, kind) + r1cs.num_public(s) + 1
    _SHARED["a"] = a
    if workers <= 1:
        parts = [_row_sums((s, kind, zp, toxic.tau, n_dom, 0, nrows))]
    else:
        import multiprocessing as mp
        step = -(-nrows // (workers * 4))
        jobs = [(s, kind, zp, toxic.tau, n_dom, c, min(c + step, nrows)) for c in range(0, nrows, step)]
        with mp.get_context("fork").Pool(workers) as pool:
            parts = pool.map(_row_sums, jobs)
    _SHARED.clear()
    At, Bt, Ct, Aw, Bw, Cw = (sum(p[q] for p in parts) % R for q in range(6))
    d_inv = _inv(toxic.delta)
    msm_l = (toxic.beta * Aw + toxic.alpha * Bw + Cw) * d_inv % R
    msm_h = (At * Bt - Ct) * d_inv % R
    a_A = (toxic.alpha + At + r * toxic.delta) % R
    b_B = (toxic.beta + Bt + s_rand * toxic.delta) % R
    c_C = (msm_l + msm_h + s_rand * a_A + r * b_B - r * s_rand * toxic.delta) % R
    return {"A": a_A, "B": b_B, "C": c_C, "msm_A": At, "msm_B": Bt, "msm_L": msm_l,
            "msm_H": msm_h, "Y": Y}


def expected_proof_trapdoor(s, kind, toxic, X, W, r, s_rand, z=None, workers=1):
    t = trapdoor_scalars(s, kind, toxic, X, W, r, s_rand, z, workers)
    return Proof(g1_mul(G1_GEN, t["A"]), g2_mul(G2_GEN, t["B"]), g1_mul(G1_GEN, t["C"])), t["Y"]
