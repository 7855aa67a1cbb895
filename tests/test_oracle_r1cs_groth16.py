"""Pins for the oracle's constraint systems and Groth16 (no GPU).

The CRPC and PSQ builders are pinned to the paper's worked examples
(tests/golden/*.json, each with its citation) and to symbolic polynomial
identities; Groth16 is pinned by the pairing verification equation, which is
independent of how the prover computed its proof, and by tamper tests.
"""
import json
import os
import random

import pytest

import synth
from oracle import bn254 as bn
from oracle import encoding, groth16, qap, r1cs
from oracle.bn254 import R

ALL_KINDS = (r1cs.PLAIN, r1cs.CRPC_PSQ, r1cs.PLAIN_ADD, r1cs.PLAIN_PSQ, r1cs.CRPC)


def _inputs(seed, a, n, b):
    X, W = synth.matmul_inputs(seed, a, n, b)
    return X.astype(int).tolist(), W.astype(int).tolist()


# ----------------------------------------------------------------------------
# polynomial helpers in a formal variable Z over the integers (dict: exp -> coeff)
def _padd(p, q):
    out = dict(p)
    for e, c in q.items():
        out[e] = out.get(e, 0) + c
    return {e: c for e, c in out.items() if c}


def _pmul(p, q):
    out = {}
    for e1, c1 in p.items():
        for e2, c2 in q.items():
            out[e1 + e2] = out.get(e1 + e2, 0) + c1 * c2
    return {e: c for e, c in out.items() if c}


def test_crpc_worked_example_layout(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "crpc_worked_example.json")))
    s = r1cs.Shape(g["a"], g["n"], g["b"])
    # the builder's exponents for each entry, read off the CRPC rows at a
    # "z" that encodes exponents: compare z^e against z powers
    z = 7
    zp = {pow(z, e, R): e for e in range(s.a * s.b)}
    rows = list(r1cs.rows(s, r1cs.CRPC_PSQ, z))
    for k in range(s.n):
        A, B, _ = rows[k]
        for key, e in g["x_exponents_by_column"][str(k)].items():
            i, kk = int(key[0]), int(key[1])
            assert kk == k and zp[A[r1cs.var_x(s, i, k)]] == e
        for key, e in g["w_exponents_by_row"][str(k)].items():
            kk, j = int(key[0]), int(key[1])
            assert kk == k and zp[B[r1cs.var_w(s, k, j)]] == e
    _, _, C_last = rows[s.n - 1]
    for key, e in g["y_exponents"].items():
        i, j = int(key[0]), int(key[1])
        assert zp[C_last[r1cs.var_y(s, i, j)]] == e
    assert r1cs.num_constraints(s, r1cs.PLAIN) == g["vanilla_multiplication_constraints"]
    assert r1cs.num_constraints(s, r1cs.CRPC_PSQ) == g["crpc_multiplication_constraints"]


@pytest.mark.parametrize("shape", [(3, 2, 2), (2, 3, 4), (4, 5, 3), (1, 6, 7)])
def test_crpc_identity_symbolic(shape):
    """Coefficient of Z^(ib+j) in sum_k X_k(Z) W_k(Z) is exactly y_ij, as integers."""
    a, n, b = shape
    X, W = _inputs(sum(shape), a, n, b)
    Y = r1cs.matmul(X, W)
    total = {}
    for k in range(n):
        Xk = {i * b: X[i][k] for i in range(a) if X[i][k]}
        Wk = {j: W[k][j] for j in range(b) if W[k][j]}
        total = _padd(total, _pmul(Xk, Wk))
    want = {i * b + j: Y[i][j] for i in range(a) for j in range(b) if Y[i][j]}
    assert total == want


def test_sum_of_outputs_transform_is_unsound_but_crpc_is_not():
    """Section III-A's first transform accepts a wrong Y; the CRPC rows reject it."""
    s = r1cs.Shape(3, 2, 2)
    X, W = _inputs(5, 3, 2, 2)
    Y = r1cs.matmul(X, W)
    bad = [row[:] for row in Y]
    bad[0][0] += 1
    bad[2][1] -= 1
    lhs = sum(sum(row) for row in bad)
    rhs = sum(sum(X[i][k] for i in range(3)) * sum(W[k][j] for j in range(2)) for k in range(2))
    assert lhs == rhs  # the summed check is fooled
    z = synth.crpc_point(5)
    a, _ = r1cs.assignment(s, r1cs.CRPC_PSQ, X, W, z)
    for t, v in enumerate(y for row in bad for y in row):
        a[r1cs.var_y(s, 0, 0) + t] = v % R
    assert not r1cs.is_satisfied(s, r1cs.CRPC_PSQ, a, z)


def test_misaligned_transform_has_cross_terms():
    """Section III-A's single-product transform leaves terms that belong to no y_ij."""
    x = {(0, 0): 1, (0, 1): 0, (1, 0): 5, (1, 1): 4, (2, 0): 9, (2, 1): 8}
    w = {(0, 0): 0, (0, 1): 2, (1, 0): 1, (1, 1): 3}
    # symbolic: variables as generators, track which (x, w) pair lands on each exponent
    prod = {}
    for xv, ex in x.items():
        for wv, ew in w.items():
            prod.setdefault(ex + ew, []).append((xv, wv))
    y_exp = {(0, 0): 1, (0, 1): 3, (1, 0): 5, (1, 1): 7, (2, 0): 9, (2, 1): 11}
    wanted = {(i, j): {((i, k), (k, j)) for k in range(2)} for i in range(3) for j in range(2)}
    cross = 0
    for e, pairs in prod.items():
        owner = [ij for ij, ye in y_exp.items() if ye == e]
        for pair in pairs:
            if not owner or pair not in wanted[owner[0]]:
                cross += 1
    assert cross > 0
    # With the exponents as printed, the term at Z^0 is x01 w00, which belongs
    # to no output (the text names x01 w01 there; that product lands on Z^2).
    assert prod[0] == [((0, 1), (0, 0))]


def test_psq_worked_example_counts(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "psq_worked_example.json")))
    s = r1cs.Shape(g["a"], g["n"], g["b"])
    assert r1cs.num_constraints(s, r1cs.PLAIN_ADD) == g["long_addition"]["constraints"]
    assert len(r1cs.left_wire_variables(s, r1cs.PLAIN_ADD)) == g["long_addition"]["left_wire_variables"]
    assert r1cs.num_constraints(s, r1cs.PLAIN_PSQ) == g["prefix_sum"]["constraints"]
    assert len(r1cs.left_wire_variables(s, r1cs.PLAIN_PSQ)) == g["prefix_sum"]["left_wire_variables"]
    # PSQ's last prefix sum is the dot product itself
    X, W = [[3, -2, 5]], [[4], [7], [-1]]
    a, Y = r1cs.assignment(s, r1cs.PLAIN_PSQ, X, W)
    aux = a[r1cs.var_aux(s, 0):]
    assert aux == [12, (12 - 14) % R]
    assert Y == [[3 * 4 - 2 * 7 - 5]]


@pytest.mark.parametrize("kind", ALL_KINDS)
def test_counts_and_satisfaction(kind):
    s = r1cs.Shape(3, 4, 5)
    X, W = _inputs(2, 3, 4, 5)
    z = synth.crpc_point(2) if kind in r1cs.CRPC_KINDS else None
    a, Y = r1cs.assignment(s, kind, X, W, z)
    assert len(a) == r1cs.num_vars(s, kind)
    assert r1cs.is_satisfied(s, kind, a, z)
    assert sum(1 for _ in r1cs.rows(s, kind, z)) == r1cs.num_constraints(s, kind) + r1cs.num_public(s) + 1
    want_m = {r1cs.PLAIN: 60, r1cs.PLAIN_PSQ: 60, r1cs.PLAIN_ADD: 75, r1cs.CRPC_PSQ: 4, r1cs.CRPC: 5}
    assert r1cs.num_constraints(s, kind) == want_m[kind]
    # a wrong output breaks satisfaction
    a[r1cs.var_y(s, 1, 2)] = (a[r1cs.var_y(s, 1, 2)] + 1) % R
    assert not r1cs.is_satisfied(s, kind, a, z)


def test_crpc_psq_last_prefix_is_y_of_z():
    s = r1cs.Shape(4, 6, 3)
    X, W = _inputs(9, 4, 6, 3)
    z = synth.crpc_point(9)
    a, Y = r1cs.assignment(s, r1cs.CRPC, X, W, z)
    yz = sum(pow(z, i * s.b + j, R) * Y[i][j] for i in range(s.a) for j in range(s.b)) % R
    prods = a[r1cs.var_aux(s, 0):]
    assert sum(prods) % R == yz
    a2, _ = r1cs.assignment(s, r1cs.CRPC_PSQ, X, W, z)
    pre = a2[r1cs.var_aux(s, 0):]
    assert pre == [sum(prods[:k + 1]) % R for k in range(s.n - 1)]


def test_paper_shape_sizes():
    s = r1cs.Shape(49, 320, 512)
    assert r1cs.num_public(s) == 40768
    assert r1cs.num_constraints(s, r1cs.PLAIN) == 8028160
    assert r1cs.domain_size(s, r1cs.PLAIN) == 1 << 23
    assert r1cs.domain_size(s, r1cs.CRPC_PSQ) == 1 << 16
    assert r1cs.num_vars(s, r1cs.CRPC_PSQ) == 204928
    assert r1cs.num_vars(s, r1cs.PLAIN) == 8207681
    toy = r1cs.Shape(4, 8, 4)
    assert r1cs.num_constraints(toy, r1cs.PLAIN) == 128 and r1cs.domain_size(toy, r1cs.PLAIN) == 256


def test_var_polys_interpolate_rows():
    """u_i(omega^c) = A[c][i]: checked through the product-form Lagrange basis."""
    s = r1cs.Shape(2, 3, 2)
    z = 11
    for kind in (r1cs.PLAIN, r1cs.CRPC_PSQ):
        n_dom = r1cs.domain_size(s, kind)
        tau = 123456789123456789
        u, v, w = qap.var_polys_at(s, kind, tau, z)
        Lp = qap.lagrange_basis_at_product_form(n_dom, tau)
        u2 = [0] * len(u)
        for c, (A, _, _) in enumerate(r1cs.rows(s, kind, z)):
            for i, coef in A.items():
                u2[i] = (u2[i] + coef * Lp[c]) % R
        assert u == u2


# ----------------------------------------------------------------------------
# Groth16
@pytest.fixture(scope="module")
def toy_keys():
    s = r1cs.Shape(2, 3, 2)
    tox = groth16.Toxic(*synth.toxic_waste(3))
    z = synth.crpc_point(3)
    out = {}
    for kind in ALL_KINDS:
        zz = z if kind in r1cs.CRPC_KINDS else None
        out[kind] = groth16.setup(s, kind, tox, zz)
    return s, tox, z, out


@pytest.mark.slow
@pytest.mark.parametrize("kind", ALL_KINDS)
def test_groth16_complete_and_matches_trapdoor(toy_keys, kind):
    s, tox, z, keys = toy_keys
    pk, vk = keys[kind]
    zz = z if kind in r1cs.CRPC_KINDS else None
    X, W = _inputs(4, s.a, s.n, s.b)
    r, sr = synth.prover_randomness(4)
    proof, Y = groth16.prove(pk, X, W, r, sr)
    assert groth16.verify(vk, X, Y, proof)
    want, _ = groth16.expected_proof_trapdoor(s, kind, tox, X, W, r, sr, zz)
    assert bn.g1_eq(proof.A, want.A) and bn.g2_eq(proof.B, want.B) and bn.g1_eq(proof.C, want.C)
    # schoolbook quotient gives the same proof
    proof2, _ = groth16.prove(pk, X, W, r, sr, quotient="schoolbook")
    assert proof2 == proof
    # vk blob round trip
    vk2 = encoding.vk_from_blob(encoding.vk_blob(vk))
    assert encoding.vk_blob(vk2) == encoding.vk_blob(vk)
    assert encoding.proof_from(encoding.proof_bytes(proof)) == tuple(proof)


@pytest.mark.slow
def test_groth16_rejects_tampering(toy_keys):
    s, tox, z, keys = toy_keys
    pk, vk = keys[r1cs.CRPC_PSQ]
    X, W = _inputs(6, s.a, s.n, s.b)
    r, sr = synth.prover_randomness(6)
    proof, Y = groth16.prove(pk, X, W, r, sr)
    assert groth16.verify(vk, X, Y, proof)
    Xb = [row[:] for row in X]
    Xb[1][2] += 1
    assert not groth16.verify(vk, Xb, Y, proof)
    Yb = [row[:] for row in Y]
    Yb[0][1] -= 1
    assert not groth16.verify(vk, X, Yb, proof)
    g = bn.G1_GEN
    assert not groth16.verify(vk, X, Y, groth16.Proof(bn.g1_add(proof.A, g), proof.B, proof.C))
    assert not groth16.verify(vk, X, Y, groth16.Proof(proof.A, bn.g2_add(proof.B, bn.G2_GEN), proof.C))
    assert not groth16.verify(vk, X, Y, groth16.Proof(proof.A, proof.B, bn.g1_add(proof.C, g)))
    assert not groth16.verify(vk, X, Y, groth16.Proof(None, proof.B, proof.C))
    assert not groth16.verify(vk, X, Y, groth16.Proof((1, 3), proof.B, proof.C))
    # a proof for other inputs does not verify this statement
    X2, W2 = _inputs(7, s.a, s.n, s.b)
    proof2, Y2 = groth16.prove(pk, X2, W2, r, sr)
    assert groth16.verify(vk, X2, Y2, proof2)
    assert not groth16.verify(vk, X, Y, proof2)


def test_trapdoor_localizes_msms():
    """Per-MSM trapdoor values are consistent with the proof scalars."""
    s = r1cs.Shape(2, 2, 2)
    tox = groth16.Toxic(*synth.toxic_waste(8))
    X, W = _inputs(8, 2, 2, 2)
    r, sr = synth.prover_randomness(8)
    t = groth16.trapdoor_scalars(s, r1cs.PLAIN, tox, X, W, r, sr)
    assert t["A"] == (tox.alpha + t["msm_A"] + r * tox.delta) % R
    assert t["B"] == (tox.beta + t["msm_B"] + sr * tox.delta) % R
    assert t["C"] == (t["msm_L"] + t["msm_H"] + sr * t["A"] + r * t["B"] - r * sr * tox.delta) % R


def test_parallel_and_sampled_sums_match_serial():
    """The process-split trapdoor and the sampled u/v/w agree with the serial definitions."""
    s = r1cs.Shape(3, 5, 4)
    tox = groth16.Toxic(*synth.toxic_waste(21))
    z = synth.crpc_point(21)
    X, W = _inputs(21, 3, 5, 4)
    r, sr = synth.prover_randomness(21)
    for kind in ALL_KINDS:
        zz = z if kind in r1cs.CRPC_KINDS else None
        t1 = groth16.trapdoor_scalars(s, kind, tox, X, W, r, sr, zz, workers=1)
        t2 = groth16.trapdoor_scalars(s, kind, tox, X, W, r, sr, zz, workers=3)
        assert t1 == t2
        u, v, w = qap.var_polys_at(s, kind, tox.tau, zz)
        sample = [0, 1, 7, r1cs.num_vars(s, kind) - 1]
        got = qap.var_polys_sampled(s, kind, tox.tau, sample, zz, workers=2)
        assert got == {i: (u[i], v[i], w[i]) for i in sample}
