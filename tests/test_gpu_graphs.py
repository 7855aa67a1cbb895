"""Graph replay of repeated proofs (zkvc_set_graphs) against eager launches and the oracle.

Bar: bit-exact.  The second call of a composition in a row on a context is
captured into a HIP graph and later calls replay it with X and W restaged, so
every call from the third on is a replay.  Each proof must equal the oracle's
closed-form trapdoor proof and the eager proof of the same inputs, with other
device work and host synchronizations between the replays, and after the
composition changes and comes back.
"""
import numpy as np
import pytest

import synth
from oracle import groth16, r1cs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def zk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_12217_amd import zkvc
    zkvc.lib()
    prev = zkvc.set_graphs(1)
    yield zkvc
    zkvc.set_graphs(prev)


@pytest.fixture(scope="module")
def keys(zk):
    # the last shape has a domain of 2^11 (three NTT passes with small tiles)
    specs = [((4, 8, 4), r1cs.CRPC_PSQ, 11), ((3, 5, 6), r1cs.PLAIN, 12), ((5, 24, 9), r1cs.PLAIN, 13)]
    out = []
    for shape, kind, seed in specs:
        tox = groth16.Toxic(*synth.toxic_waste(seed))
        z = synth.crpc_point(seed) if kind in r1cs.CRPC_KINDS else None
        out.append((shape, kind, tox, z, zk.setup(*shape, kind, tuple(tox), z)))
    yield out
    for *_, pk in out:
        pk.close()


def _inputs(key, seed, job):
    (a, n, b), *_ = key
    X, W = synth.matmul_inputs(seed, a, n, b)
    r, s = synth.prover_randomness(seed, job=job)
    return X, W, r, s


def _expected(key, X, W, r, s):
    (a, n, b), kind, tox, z, _ = key
    proof, Y = groth16.expected_proof_trapdoor(r1cs.Shape(a, n, b), kind, tox, X.astype(int).tolist(),
                                                W.astype(int).tolist(), r, s, z)
    return tuple(proof), Y


def _device_noise():
    """Unrelated eager device work and a host synchronization."""
    x = torch.arange(1 << 20, device="cuda", dtype=torch.int64)
    assert int((x * 3 + 1).sum().item()) == 3 * ((1 << 20) * ((1 << 20) - 1) // 2) + (1 << 20)
    torch.cuda.synchronize()


def test_single_proof_replays(zk, keys):
    """Five rounds over three keys (each key's own context): capture, then replays."""
    done = []
    for it in range(5):
        for ki, key in enumerate(keys):
            X, W, r, s = _inputs(key, 300 + 10 * it + ki, ki)
            Y, proof = zk.prove(key[4], X, W, r, s)
            want, Yo = _expected(key, X, W, r, s)
            assert Y.tolist() == Yo, (it, ki)
            assert zk.proof_to_tuple(proof) == want, (it, ki)
            st = key[4].last_stats()
            assert st.total_ms > 0 and st.witness_ms >= 0 and st.msm_ms >= 0
            done.append((ki, X, W, r, s, Y, zk.proof_bytes(proof)))
        _device_noise()
    # the same inputs proven eagerly give the same bytes
    prev = zk.set_graphs(0)
    try:
        for ki, X, W, r, s, Y, pb in done:
            Y0, p0 = zk.prove(keys[ki][4], X, W, r, s)
            assert np.array_equal(Y0, Y) and zk.proof_bytes(p0) == pb
    finally:
        zk.set_graphs(prev)


def test_batch_replays_across_composition_changes(zk, keys):
    """Batch compositions c1 c1 c1 c2 c1 c1 c1: capture, replay, invalidation, recapture."""
    c1 = [0, 2, 1, 0]
    c2 = [1, 1]
    for it, comp in enumerate([c1, c1, c1, c2, c1, c1, c1]):
        jobs = [(keys[ki], *_inputs(keys[ki], 500 + 16 * it + q, q)) for q, ki in enumerate(comp)]
        got = zk.prove_batch([(key[4], X, W, r, s) for key, X, W, r, s in jobs])
        for q, ((key, X, W, r, s), (Y, proof)) in enumerate(zip(jobs, got)):
            want, Yo = _expected(key, X, W, r, s)
            assert Y.tolist() == Yo, (it, q)
            assert zk.proof_to_tuple(proof) == want, (it, q)
        if it % 2:
            _device_noise()


def test_switch_off_and_on(zk, keys):
    """Turning replay off and on between calls of one composition."""
    key = keys[0]
    for it, flag in enumerate([1, 1, 0, 1, 1, 0, 0, 1, 1, 1]):
        zk.set_graphs(flag)
        X, W, r, s = _inputs(key, 700 + it, 0)
        Y, proof = zk.prove(key[4], X, W, r, s)
        want, Yo = _expected(key, X, W, r, s)
        assert Y.tolist() == Yo and zk.proof_to_tuple(proof) == want, it
    zk.set_graphs(1)
