"""Host-side Spartan checks (no GPU): the library's instance sizes equal the
oracle's, and the library's host verifier accepts the oracle's proofs and
rejects changed ones (the verifier makes no device call)."""
import os

import pytest

import synth
from oracle import bn254 as bn
from oracle import r1cs, spartan as sp


@pytest.fixture(scope="module")
def zk():
    from paper_2504_12217_amd import zkvc
    if not os.path.exists(zkvc.LIB_PATH):
        pytest.skip("library not built")
    zkvc.lib()
    return zkvc


@pytest.mark.parametrize("a,n,b,kind", [(2, 3, 2, 1), (49, 320, 512, 1), (49, 64, 128, 4), (1, 1, 1, 1), (7, 1, 9, 4)])
def test_sizes_match_oracle(zk, a, n, b, kind):
    inst = sp.Instance(r1cs.Shape(a, n, b), kind, 3)
    info = zk.spartan_info(a, n, b, kind)
    assert (info.constraints, info.sx, info.sy, info.rows, info.cols) == (inst.m, inst.sx, inst.sy, inst.rows,
                                                                           inst.cols)
    assert info.proof_bytes == inst.rows * 64 + (4 * inst.sx + 3 + 3 * inst.sy + inst.cols) * 32


class _Key:
    """The library's verifier through a key-like wrapper without device state."""

    def __init__(self, zk, shape, kind, z, gens):
        self.zk, self.shape, self.kind, self.z, self.gens = zk, shape, kind, z, gens

    def verify(self, X, Y, proof):
        import ctypes
        import numpy as np
        zk = self.zk
        X = np.ascontiguousarray(X, dtype=np.int8)
        Y = np.ascontiguousarray(Y, dtype=np.int32)
        g = zk._g1_array(self.gens)
        pb = (ctypes.c_uint8 * len(proof)).from_buffer_copy(proof)
        return zk.lib().zkvc_spartan_verify(ctypes.byref(zk.Shape(*self.shape, self.kind)), ctypes.byref(zk.fr(self.z)),
                                            ctypes.cast(g, ctypes.c_void_p), len(self.gens), X.ctypes.data,
                                            Y.ctypes.data, ctypes.cast(pb, ctypes.c_void_p), len(proof))


@pytest.mark.parametrize("shape,kind", [((2, 3, 2), r1cs.CRPC_PSQ), ((3, 4, 2), r1cs.CRPC), ((1, 2, 3), r1cs.CRPC_PSQ)])
def test_library_verifier_on_oracle_proofs(zk, shape, kind):
    z = 23 + kind
    inst = sp.Instance(r1cs.Shape(*shape), kind, z)
    gens = [bn.g1_mul(bn.G1_GEN, k) for k in synth.nonzero_fr(3, synth.STREAM_MSM_BASES, inst.cols)]
    X, W = synth.matmul_inputs(11, *shape)
    Xl, Wl = X.astype(int).tolist(), W.astype(int).tolist()
    proof, Y = sp.prove(inst, Xl, Wl, gens)
    data = sp.proof_bytes(proof)
    key = _Key(zk, shape, kind, z, gens)
    assert key.verify(X, Y, data) == 1
    bad = [row[:] for row in Y]
    bad[0][0] += 1
    assert key.verify(X, bad, data) == 0
    for pos in (3, inst.rows * 64 + 40, len(data) - 40, len(data) - 1):
        flipped = bytearray(data)
        flipped[pos] ^= 0x10
        assert key.verify(X, Y, bytes(flipped)) == 0, pos
    assert key.verify(X, Y, data + b"\x00") == 0
    other = _Key(zk, shape, kind, z + 1, gens)
    assert other.verify(X, Y, data) == 0
