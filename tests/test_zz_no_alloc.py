"""zkvc_msm_g1_noalloc (the allocation-free MSM) against zkvc_msm_g1.

Two calls in a row on the fixed scratch, the second with a smaller input
(the array keeps the first call's contents), each compared bit for bit with
zkvc_msm_g1 on the same inputs and with the discrete-log identity
sum s_i [k_i]G = [sum s_i k_i mod r]G; then the largest accepted size, the
internal layout, and the rejection of a size beyond the limit (decided
before anything is launched).
"""
import numpy as np
import pytest

import synth
from oracle import bn254 as bn
from tests.gpu_util import dev_words

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MAX_N = 1 << 16


@pytest.fixture(scope="module")
def zk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_12217_amd import zkvc
    zkvc.lib()
    return zkvc


def _case(zk, n, seed):
    ks = synth.fr_limbs(seed, synth.STREAM_MSM_BASES, n)
    sc = synth.fr_limbs(seed, synth.STREAM_MSM_SCALARS, n)
    pts = torch.zeros((n * 16,), dtype=torch.int32, device="cuda")
    zk.fixed_base_g1(dev_words(ks), n, pts)
    want = bn.g1_mul(bn.G1_GEN, sum(a * b for a, b in zip(synth.limbs_to_ints(ks), synth.limbs_to_ints(sc))) % bn.R)
    return pts, dev_words(sc), want


def test_two_calls_in_a_row_second_smaller(zk):
    for n, seed in ((40000, 71), (777, 72)):
        pts, sc, want = _case(zk, n, seed)
        got = zk.msm_g1_noalloc(pts, sc, n)
        assert got == zk.msm_g1(pts, sc, n), n
        assert got == want, n


def test_largest_size_and_internal_layout(zk):
    pts, sc, want = _case(zk, MAX_N, 73)
    assert zk.msm_g1_noalloc(pts, sc, MAX_N) == want
    # the same points and scalars in the internal (Montgomery) layout
    pm = torch.zeros_like(pts)
    zk.field_op(zk.FQ, zk.OP_TO_MONT, pts, None, pm, 2 * MAX_N)
    sm = torch.zeros_like(sc)
    zk.field_op(zk.FR, zk.OP_TO_MONT, sc, None, sm, MAX_N)
    assert zk.msm_g1_noalloc(pm, sm, MAX_N, flags=zk.LAYOUT_MONT) == want
    assert zk.msm_g1(pm, sm, MAX_N, flags=zk.LAYOUT_MONT) == want
    # a small call after the largest one
    pts2, sc2, want2 = _case(zk, 5, 74)
    assert zk.msm_g1_noalloc(pts2, sc2, 5) == want2 == zk.msm_g1(pts2, sc2, 5)


def test_edge_cases_and_rejection(zk):
    d = dev_words(np.zeros((4, 16), dtype=np.uint32))
    assert zk.msm_g1_noalloc(d, d, 0) is None
    with pytest.raises(zk.ZkvcError) as e:
        zk.msm_g1_noalloc(d, d, MAX_N + 1)
    assert e.value.code == zk.EINVAL and "65536" in str(e.value)
    with pytest.raises(zk.ZkvcError) as e:
        zk.msm_g1_noalloc(d, d, 2, flags=8)
    assert e.value.code == zk.EINVAL
    # duplicate bases, P and -P, an infinity base, scalars 0, 1 and r - 1
    g = bn.G1_GEN
    P1, P2 = bn.g1_mul(g, 11), bn.g1_mul(g, 29)
    pts = [P1, P1, P2, bn.g1_neg(P2), None, P1]
    sc = [5, 5, 9, 9, 3, bn.R - 1]
    words = []
    for p in pts:
        words += [0, 0] if p is None else [p[0], p[1]]
    dp = dev_words(synth.ints_to_limbs(words).reshape(-1, 16))
    ds = dev_words(synth.ints_to_limbs(sc))
    assert zk.msm_g1_noalloc(dp, ds, len(pts)) == bn.g1_msm(pts, sc) == zk.msm_g1(dp, ds, len(pts))
