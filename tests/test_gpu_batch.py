"""Batched proving (zkvc_prove_batch) against single proofs and the oracle.

Bar: bit-exact.  A proof is unique for fixed (key, X, W, r, s), so every proof
of a batch must equal the single proof of the same job, and the oracle's
closed-form trapdoor proof, whatever else shares the batch: shapes, kinds,
repeated keys, several proofs of one domain size (the table-driven batched
quotient) or one alone.
"""
import numpy as np
import pytest

import synth
from oracle import bn254, groth16, r1cs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def zk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_12217_amd import zkvc
    zkvc.lib()
    return zkvc


@pytest.fixture(scope="module")
def keys(zk):
    """Proving keys of several shapes and kinds (seeded toxic waste per key)."""
    specs = [((4, 8, 4), r1cs.PLAIN, 1), ((4, 8, 4), r1cs.CRPC_PSQ, 2), ((3, 5, 6), r1cs.CRPC_PSQ, 3),
             ((2, 7, 3), r1cs.PLAIN_PSQ, 4), ((5, 4, 2), r1cs.CRPC, 5), ((3, 3, 3), r1cs.PLAIN_ADD, 6)]
    out = []
    for shape, kind, seed in specs:
        tox = groth16.Toxic(*synth.toxic_waste(seed))
        z = synth.crpc_point(seed) if kind in r1cs.CRPC_KINDS else None
        out.append((shape, kind, tox, z, zk.setup(*shape, kind, tuple(tox), z)))
    yield out
    for *_, pk in out:
        pk.close()


def _jobs(keys, order, base_seed):
    """(key index, X, W, r, s) per job; inputs from a seed per job."""
    jobs = []
    for q, ki in enumerate(order):
        (a, n, b), *_ = keys[ki]
        X, W = synth.matmul_inputs(base_seed + q, a, n, b)
        r, s = synth.prover_randomness(base_seed, job=q)
        jobs.append((ki, X, W, r, s))
    return jobs


def _expected(keys, job):
    ki, X, W, r, s = job
    (a, n, b), kind, tox, z, _ = keys[ki]
    proof, Y = groth16.expected_proof_trapdoor(r1cs.Shape(a, n, b), kind, tox, X.astype(int).tolist(),
                                                W.astype(int).tolist(), r, s, z)
    return tuple(proof), Y


def _run_and_check(zk, keys, jobs):
    got = zk.prove_batch([(keys[ki][4], X, W, r, s) for ki, X, W, r, s in jobs])
    assert len(got) == len(jobs)
    for job, (Y, proof) in zip(jobs, got):
        ki, X, W, r, s = job
        want, Yo = _expected(keys, job)
        assert Y.tolist() == Yo
        assert zk.proof_to_tuple(proof) == want
        # the single proof of the same job is the same
        Y1, p1 = zk.prove(keys[ki][4], X, W, r, s)
        assert np.array_equal(Y1, Y) and zk.proof_bytes(p1) == zk.proof_bytes(proof)
        assert zk.verify(keys[ki][4].vk, X, Y, proof) == 1


def test_batch_mixed_shapes_and_kinds(zk, keys):
    _run_and_check(zk, keys, _jobs(keys, [0, 1, 2, 3, 4, 5], 100))


def test_batch_repeated_keys_share_quotient_launches(zk, keys):
    # several proofs per key: each domain size has a group of several proofs
    _run_and_check(zk, keys, _jobs(keys, [1, 1, 0, 2, 1, 0, 3, 3, 4, 5, 5], 200))


def test_batch_of_one_equals_single(zk, keys):
    _run_and_check(zk, keys, _jobs(keys, [2], 300))


def test_batch_context_reused_with_other_sizes(zk, keys):
    # a larger batch, then a smaller one of other keys, on the same stream
    _run_and_check(zk, keys, _jobs(keys, [0, 1, 2, 3, 4, 5, 0, 1, 2], 400))
    _run_and_check(zk, keys, _jobs(keys, [4, 3], 500))


def test_batch_argument_errors(zk, keys):
    pk = keys[0][4]
    X, W = synth.matmul_inputs(7, 4, 8, 4)
    with pytest.raises(zk.ZkvcError) as e:
        zk.prove_batch([(pk, X, W, bn254.R, 1)])  # r out of range
    assert e.value.code == zk.EINVAL
    assert zk.lib().zkvc_prove_batch(None, 0, None) == zk.EINVAL
    with pytest.raises(ValueError):
        zk.prove_batch([(pk, X[:, :3], W, 1, 2)])
