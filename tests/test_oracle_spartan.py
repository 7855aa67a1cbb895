"""Pins of the oracle's Spartan backend (zkVC-S, Section II and Table II).

Each piece is checked against what the mathematics fixes, not against a
retyping of itself: multilinear extensions agree with their tables on the
Boolean hypercube and are affine in every coordinate; the eq table sums to
one; round polynomials interpolate exactly; the first sum-check's claim is
zero exactly when the R1CS is satisfied (brute force over the hypercube);
the dense M vector and the verifier's sparse evaluation of the matrices'
extension agree; and proofs are complete for every circuit kind and
rejected when any part, or the statement, is changed.
"""
import random

import pytest

import synth
from oracle import bn254 as bn
from oracle import r1cs, spartan as sp
from oracle.bn254 import R

SHAPES = [(r1cs.Shape(2, 3, 2), k) for k in (r1cs.CRPC_PSQ, r1cs.CRPC, r1cs.PLAIN, r1cs.PLAIN_PSQ, r1cs.PLAIN_ADD)]


def _gens(inst, seed=5):
    ks = synth.nonzero_fr(seed, synth.STREAM_MSM_BASES, inst.cols)
    return [bn.g1_mul(bn.G1_GEN, k) for k in ks]


def _inputs(s, seed):
    X, W = synth.matmul_inputs(seed, s.a, s.n, s.b)
    return X.astype(int).tolist(), W.astype(int).tolist()


def test_multilinear_extension_on_hypercube_and_affine():
    rng = random.Random(1)
    f = [rng.randrange(R) for _ in range(16)]
    for i in range(16):
        assert sp.mle_eval(f, [(i >> k) & 1 for k in range(4)]) == f[i]
    r = [rng.randrange(R) for _ in range(4)]
    # affine in the first coordinate: f~(c, rest) = (1 - c) f~(0, rest) + c f~(1, rest)
    v0 = sp.mle_eval(f, [0] + r[1:])
    v1 = sp.mle_eval(f, [1] + r[1:])
    assert sp.mle_eval(f, r) == ((1 - r[0]) * v0 + r[0] * v1) % R
    # folding binds the least significant variable
    assert sp.mle_eval(sp.fold(f, r[0]), r[1:]) == sp.mle_eval(f, r)
    assert sum(sp.eq_table(r)) % R == 1


def test_interpolation_is_exact():
    rng = random.Random(2)
    coef = [rng.randrange(R) for _ in range(4)]

    def p(x):
        return sum(c * pow(x, k, R) for k, c in enumerate(coef)) % R

    x = rng.randrange(R)
    assert sp.interpolate([p(t) for t in range(4)], x) == p(x)


@pytest.mark.parametrize("s,kind", SHAPES)
def test_first_claim_is_zero_iff_satisfied(s, kind):
    z = 7 if kind in r1cs.CRPC_KINDS else None
    inst = sp.Instance(s, kind, z)
    X, W = _inputs(s, 3)
    a, _ = r1cs.assignment(s, kind, X, W, z)
    rng = random.Random(4)
    tau = [rng.randrange(R) for _ in range(inst.sx)]
    eq = sp.eq_table(tau)

    def total(assign):
        acc = 0
        for c in range(inst.m):
            A, B, C = inst.constraint(c)
            acc += eq[c] * (r1cs.dot(A, assign) * r1cs.dot(B, assign) - r1cs.dot(C, assign))
        return acc % R

    assert total(a) == 0
    bad = list(a)
    bad[-1] = (bad[-1] + 1) % R  # an auxiliary (or W) value off by one
    assert total(bad) != 0


@pytest.mark.parametrize("s,kind", SHAPES[:3])
def test_dense_m_vector_matches_sparse_matrix_extension(s, kind):
    z = 11 if kind in r1cs.CRPC_KINDS else None
    inst = sp.Instance(s, kind, z)
    rng = random.Random(5)
    rx = [rng.randrange(R) for _ in range(inst.sx)]
    ry = [rng.randrange(R) for _ in range(inst.sy)]
    ra, rb, rc = (rng.randrange(R) for _ in range(3))
    M = sp.m_vector(inst, rx, ra, rb, rc)
    assert sp.mle_eval(M, ry) == sp.matrix_eval(inst, rx, ry, ra, rb, rc)
    # and sum_y M(y) z(y) is the weighted sum of Az~, Bz~, Cz~ at r_x
    X, W = _inputs(s, 6)
    a, _ = r1cs.assignment(s, kind, X, W, z)
    zv = inst.z_vector(a)
    az = [0] * (1 << inst.sx)
    bz, cz = list(az), list(az)
    for c in range(inst.m):
        A, B, C = inst.constraint(c)
        az[c], bz[c], cz[c] = r1cs.dot(A, a), r1cs.dot(B, a), r1cs.dot(C, a)
    want = (ra * sp.mle_eval(az, rx) + rb * sp.mle_eval(bz, rx) + rc * sp.mle_eval(cz, rx)) % R
    assert sum(m * v for m, v in zip(M, zv)) % R == want


@pytest.mark.parametrize("s,kind", SHAPES)
def test_complete_for_every_kind(s, kind):
    z = 13 if kind in r1cs.CRPC_KINDS else None
    inst = sp.Instance(s, kind, z)
    gens = _gens(inst)
    X, W = _inputs(s, 7)
    proof, Y = sp.prove(inst, X, W, gens)
    assert Y == r1cs.matmul(X, W)
    assert sp.verify(inst, X, Y, proof, gens)


def test_rejects_changed_statement_or_proof():
    s, kind = r1cs.Shape(2, 4, 3), r1cs.CRPC_PSQ
    inst = sp.Instance(s, kind, 17)
    gens = _gens(inst)
    X, W = _inputs(s, 8)
    proof, Y = sp.prove(inst, X, W, gens)
    assert sp.verify(inst, X, Y, proof, gens)
    badY = [row[:] for row in Y]
    badY[1][2] += 1
    assert not sp.verify(inst, X, badY, proof, gens)
    badX = [row[:] for row in X]
    badX[0][1] ^= 1
    assert not sp.verify(inst, badX, Y, proof, gens)

    def tweak(key, mutate):
        p = {k: (list(v) if isinstance(v, list) else v) for k, v in proof.items()}
        p[key] = mutate(p[key])
        return sp.verify(inst, X, Y, p, gens)

    assert not tweak("t", lambda t: [t[0] + 1] + t[1:])
    assert not tweak("sc1", lambda g: [[g[0][0] + 1, g[0][1] - 1] + g[0][2:]] + g[1:])
    assert not tweak("sc2", lambda g: g[:-1] + [[g[-1][0], g[-1][1], g[-1][2] + 1]])
    assert not tweak("vabc", lambda v: (v[0], v[1] + 1, v[2]))
    assert not tweak("comms", lambda c: [bn.g1_add(c[0], bn.G1_GEN)] + c[1:])


def test_layout_sizes_at_paper_shape():
    inst = sp.Instance(r1cs.Shape(49, 320, 512), r1cs.CRPC_PSQ, 3)
    assert inst.m == 320 and inst.sx == 9
    assert inst.nw == 320 * 512 + 319 and inst.ell + 1 == 40769
    assert inst.sw == 18 and inst.sy == 19 and inst.rows == 512 and inst.cols == 512


def test_proof_encoding_round_trip():
    s, kind = r1cs.Shape(2, 3, 2), r1cs.CRPC
    inst = sp.Instance(s, kind, 19)
    gens = _gens(inst)
    X, W = _inputs(s, 9)
    proof, _ = sp.prove(inst, X, W, gens)
    data = sp.proof_bytes(proof)
    assert len(data) == inst.rows * 64 + (4 * inst.sx + 3 + 3 * inst.sy + inst.cols) * 32
    back = sp.proof_from_bytes(inst, data)
    assert back["comms"] == proof["comms"] and back["t"] == proof["t"]
    assert back["sc1"] == proof["sc1"] and back["sc2"] == proof["sc2"] and back["vabc"] == tuple(proof["vabc"])
    assert sp.proof_from_bytes(inst, data[:-1]) is None
