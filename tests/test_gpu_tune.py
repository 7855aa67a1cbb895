"""The autotuner (zkvc_autotune) picks settings that change speed only: after
tuning, MSMs and NTTs still equal the oracle bit for bit.  The tuned table is
restored to the built-in rules afterwards so later tests see the defaults."""
import pytest

import synth
from oracle import bn254 as bn
from oracle import ntt as ontt
from tests.gpu_util import dev_to_ints, dev_words

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def zk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_12217_amd import zkvc
    zkvc.lib()
    before = zkvc.tune_export()
    yield zkvc
    zero = "".join(f"{ln.split()[0]} {ln.split()[1]} 0\n" for ln in zkvc.tune_export().splitlines())
    zkvc.tune_import(zero)
    zkvc.tune_import(before)


def test_autotune_then_results_unchanged(zk):
    got = zk.autotune(zk.TUNE_MSM_G1 | zk.TUNE_MSM_G2 | zk.TUNE_NTT, 8, 11)
    # G1 and G2 each set a window and a task size per size, the NTT a pass size per size
    assert got == 2 * 4 + 2 * 4 + 4
    lines = zk.tune_export().splitlines()
    assert any(ln.startswith("msm_g1 10 ") for ln in lines) and any(ln.startswith("ntt 11 ") for ln in lines)
    # tuned MSM: dlog identity on a ragged size inside the tuned range
    n = (1 << 10) - 5
    ks = synth.fr_limbs(21, synth.STREAM_MSM_BASES, n)
    sc = synth.fr_limbs(21, synth.STREAM_MSM_SCALARS, n)
    dpts = torch.zeros((n * 16,), dtype=torch.int32, device="cuda")
    zk.fixed_base_g1(dev_words(ks), n, dpts)
    k_int, s_int = synth.limbs_to_ints(ks), synth.limbs_to_ints(sc)
    assert zk.msm_g1(dpts, dev_words(sc), n) == bn.g1_mul(bn.G1_GEN, sum(a * b for a, b in zip(k_int, s_int)) % bn.R)
    # tuned NTT equals the oracle's transform
    for log_n in (9, 11):
        x = synth.fr_limbs(22 + log_n, synth.STREAM_NTT, 1 << log_n)
        d = dev_words(x)
        zk.ntt_fr(d, log_n, 0)
        assert dev_to_ints(d) == ontt.transform(synth.limbs_to_ints(x))


def test_every_window_width_equals_dlog(zk):
    """Each window width c = 2..15 forced through the tuning table: the signed
    digits (read off s + K window by window, K = sum_w (2^(c-1) - 1) 2^(c w))
    must sum the same point.  c nw exceeds 256 bits for c = 6, 7 and 9..14, so
    the recoding's ninth word is exercised.  G2 at a few widths as well."""
    n = (1 << 12) - 7
    ks = synth.fr_limbs(31, synth.STREAM_MSM_BASES, n)
    sc = synth.fr_limbs(31, synth.STREAM_MSM_SCALARS, n)
    k_int, s_int = synth.limbs_to_ints(ks), synth.limbs_to_ints(sc)
    dk, ds = dev_words(ks), dev_words(sc)
    dpts = torch.zeros((n * 16,), dtype=torch.int32, device="cuda")
    zk.fixed_base_g1(dk, n, dpts)
    want = bn.g1_mul(bn.G1_GEN, sum(a * b for a, b in zip(k_int, s_int)) % bn.R)
    try:
        for c in range(2, 16):
            zk.tune_import(f"msm_g1 12 {c}\n")
            assert zk.msm_g1(dpts, ds, n) == want, c
    finally:
        zk.tune_import("msm_g1 12 0\n")
    m = 600
    dq = torch.zeros((m * 32,), dtype=torch.int32, device="cuda")
    zk.fixed_base_g2(dev_words(ks[:m]), m, dq)
    want2 = bn.g2_mul(bn.G2_GEN, sum(a * b for a, b in zip(k_int[:m], s_int[:m])) % bn.R)
    try:
        for c in (4, 7, 11, 14):
            zk.tune_import(f"msm_g2 10 {c}\n")
            assert zk.msm_g2(dq, dev_words(sc[:m]), m) == want2, c
    finally:
        zk.tune_import("msm_g2 10 0\n")


def test_autotune_argument_errors(zk):
    for what, lo, hi in ((8, 8, 10), (1, 3, 10), (1, 12, 10), (1, 10, 23)):
        with pytest.raises(zk.ZkvcError) as e:
            zk.autotune(what, lo, hi)
        assert e.value.code == zk.EINVAL
