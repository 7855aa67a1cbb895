"""GPU parity of the field, NTT and MSM kernels against the CPU oracle.

Every call goes through the C-ABI (zkvc_field_op, zkvc_ntt_fr, zkvc_msm_g1/g2,
zkvc_fixed_base_g1/g2).  Bar: bit-exact (all arithmetic is exact modular
arithmetic; every result is unique).
"""
import random

import numpy as np
import pytest

import synth
from oracle import bn254 as bn
from oracle import ntt as ontt
from tests.gpu_util import (dev_to_ints, dev_words, g1_points_to_words, g2_points_to_words, host_words,
                            ints_to_dev, words_to_g1_points, words_to_g2_points)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def zk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_12217_amd import zkvc
    zkvc.lib()
    return zkvc


def _edge_and_random(mod, count, seed):
    edge = [0, 1, 2, mod - 1, mod - 2, (mod - 1) // 2, (mod + 1) // 2, (1 << 253) % mod, (1 << 254) % mod,
            (1 << 261) % mod, 0xFFFFFFFF, 1 << 32, (1 << 128) - 1]
    rng = random.Random(seed)
    return edge + [rng.randrange(mod) for _ in range(count)]


@pytest.mark.parametrize("field,mod", [(0, bn.P), (1, bn.R)])
def test_field_ops_bit_exact(zk, field, mod):
    a = _edge_and_random(mod, 4000, 1 + field)
    b = list(reversed(_edge_and_random(mod, 4000, 7 + field)))
    n = len(a)
    da, db = ints_to_dev(a), ints_to_dev(b)
    out = torch.zeros_like(da)
    want = {
        zk.OP_ADD: [(x + y) % mod for x, y in zip(a, b)],
        zk.OP_SUB: [(x - y) % mod for x, y in zip(a, b)],
        zk.OP_MUL: [x * y % mod for x, y in zip(a, b)],
        zk.OP_SQR: [x * x % mod for x in a],
    }
    for op, exp in want.items():
        zk.field_op(field, op, da, db, out, n)
        torch.cuda.synchronize()
        assert dev_to_ints(out) == exp, f"op {op}"
    nz = [x for x in a if x][:500]
    dnz = ints_to_dev(nz)
    out2 = torch.zeros_like(dnz)
    zk.field_op(field, zk.OP_INV, dnz, None, out2, len(nz))
    assert dev_to_ints(out2) == [pow(x, -1, mod) for x in nz]
    # internal layout round trip and its definition x * 2^261 mod m
    zk.field_op(field, zk.OP_TO_MONT, da, None, out, n)
    assert dev_to_ints(out) == [x * (1 << 261) % mod for x in a]
    back = torch.zeros_like(da)
    zk.field_op(field, zk.OP_FROM_MONT, out, None, back, n)
    assert dev_to_ints(back) == a


def _ntt_case(zk, log_n, flags, seed):
    n = 1 << log_n
    x = synth.fr_limbs(seed, synth.STREAM_NTT, n)
    d = dev_words(x)
    zk.ntt_fr(d, log_n, flags)
    torch.cuda.synchronize()
    return synth.limbs_to_ints(x), dev_to_ints(d)


@pytest.mark.parametrize("log_n", list(range(0, 13)) + [14])
@pytest.mark.parametrize("flags", [0, 1, 2, 3])
def test_ntt_matches_oracle(zk, log_n, flags):
    xs, got = _ntt_case(zk, log_n, flags, 100 + log_n)
    want = ontt.transform(xs, inverse=bool(flags & 1), coset=bool(flags & 2))
    assert got == want


@pytest.mark.parametrize("log_n", [16, 17])
def test_ntt_full_size_oracle(zk, log_n):
    xs, got = _ntt_case(zk, log_n, 0, 7)
    assert got == ontt.transform(xs)


@pytest.mark.parametrize("log_n", [20, 23])
def test_ntt_large_freivalds_and_round_trip(zk, log_n):
    n = 1 << log_n
    x = synth.fr_limbs(3, synth.STREAM_NTT, n)
    d = dev_words(x)
    zk.ntt_fr(d, log_n, 0)
    X = dev_to_ints(d)
    xs = synth.limbs_to_ints(x)
    assert ontt.freivalds_check(xs, X, 0x1234567890ABCDEF1234567890ABCDEF)
    zk.ntt_fr(d, log_n, zk.NTT_INVERSE)
    assert np.array_equal(host_words(d).reshape(-1, 8), x)
    # coset pair round trip
    zk.ntt_fr(d, log_n, zk.NTT_COSET)
    zk.ntt_fr(d, log_n, zk.NTT_COSET | zk.NTT_INVERSE)
    assert np.array_equal(host_words(d).reshape(-1, 8), x)


def test_ntt_beyond_twiddle_tables(zk):
    """2^25 points: the top pass computes its twiddles from the power tables
    (per-pass twiddle tables stop at 2^24): sampled outputs of a delta input
    against the root of unity's powers, and plain and coset round trips."""
    log_n = 25
    n = 1 << log_n
    x = np.zeros((n, 8), dtype=np.uint32)
    x[1, 0] = 1  # X_k = omega^k
    d = dev_words(x)
    zk.ntt_fr(d, log_n, 0)
    out = host_words(d).reshape(-1, 8)
    w = ontt.root_of_unity(n)
    rng = random.Random(25)
    for k in [0, 1, 2, n // 2, n - 1] + [rng.randrange(n) for _ in range(400)]:
        assert synth.limbs_to_ints(out[k:k + 1])[0] == pow(w, k, bn.R), k
    del d
    y = synth.fr_limbs(4, synth.STREAM_NTT, n)
    d = dev_words(y)
    zk.ntt_fr(d, log_n, 0)
    assert not np.array_equal(host_words(d).reshape(-1, 8), y)
    zk.ntt_fr(d, log_n, zk.NTT_INVERSE)
    assert np.array_equal(host_words(d).reshape(-1, 8), y)
    zk.ntt_fr(d, log_n, zk.NTT_COSET)
    zk.ntt_fr(d, log_n, zk.NTT_COSET | zk.NTT_INVERSE)
    assert np.array_equal(host_words(d).reshape(-1, 8), y)


def test_ntt_internal_layout_consistent(zk):
    log_n = 10
    x = synth.fr_limbs(5, synth.STREAM_NTT, 1 << log_n)
    d = dev_words(x)
    m = torch.zeros_like(d)
    zk.field_op(zk.FR, zk.OP_TO_MONT, d, None, m, 1 << log_n)
    zk.ntt_fr(m, log_n, zk.LAYOUT_MONT)
    back = torch.zeros_like(m)
    zk.field_op(zk.FR, zk.OP_FROM_MONT, m, None, back, 1 << log_n)
    zk.ntt_fr(d, log_n, 0)
    assert torch.equal(back, d)


def test_ntt_rejects_bad_arguments(zk):
    """Rejections decided before any device memory is touched."""
    d = dev_words(np.zeros((8, 8), dtype=np.uint32))
    with pytest.raises(zk.ZkvcError) as e:
        zk.ntt_fr(d, 29, 0)
    assert e.value.code == zk.EINVAL
    with pytest.raises(zk.ZkvcError):
        zk.ntt_fr(d, 3, 64)
    with pytest.raises(zk.ZkvcError):
        zk.ntt_fr(0, 3, 0)


# ------------------------------------------------------------------ MSM
def _msm_small_cases():
    rng = random.Random(42)
    g = bn.G1_GEN
    pts = [bn.g1_mul(g, rng.randrange(1, bn.R)) for _ in range(8)]
    cases = []
    for n in (1, 2, 3, 5, 8):
        cases.append((pts[:n], [rng.randrange(bn.R) for _ in range(n)]))
    cases.append(([pts[0]], [0]))
    cases.append(([pts[0]], [1]))
    cases.append(([pts[0]], [bn.R - 1]))
    cases.append(([pts[0], pts[0], pts[0]], [5, 5, 5]))                 # duplicates: bucket doubling
    cases.append(([pts[1], bn.g1_neg(pts[1])], [7, 7]))                 # P and -P cancel
    cases.append(([pts[2], None, pts[3]], [3, 9, 4]))                   # infinity base
    cases.append(([pts[4]] * 6, [rng.randrange(1 << 10) for _ in range(6)]))
    cases.append((pts, [rng.randrange(-128, 128) % bn.R for _ in range(8)]))  # int8 scalars
    cases.append((pts[:4], [bn.R - 1, bn.R - 2, (bn.R - 1) // 2, (bn.R + 1) // 2]))
    return cases


@pytest.mark.parametrize("case", range(len(_msm_small_cases())))
def test_msm_g1_small_exact(zk, case):
    pts, sc = _msm_small_cases()[case]
    dp = dev_words(g1_points_to_words(pts))
    ds = ints_to_dev(sc)
    got = zk.msm_g1(dp, ds, len(pts))
    assert got == bn.g1_msm(pts, sc)


def test_msm_g1_empty(zk):
    d = dev_words(np.zeros((1, 16), dtype=np.uint32))
    assert zk.msm_g1(d, d, 0) is None


@pytest.mark.parametrize("n", [64, 1000, 4097])
def test_msm_g1_bruteforce_medium(zk, n):
    rng = random.Random(n)
    ks = [rng.randrange(1, bn.R) for _ in range(n)]
    sc = [rng.randrange(bn.R) for _ in range(n)]
    # bases [k]G computed by the oracle; MSM checked against the discrete-log identity
    pts = [bn.g1_mul(bn.G1_GEN, k) for k in ks[:64]] if n == 64 else None
    if pts is not None:
        got = zk.msm_g1(dev_words(g1_points_to_words(pts)), ints_to_dev(sc), n)
        assert got == bn.g1_msm(pts, sc)
    else:
        dk = ints_to_dev(ks)
        dpts = torch.zeros((n * 16,), dtype=torch.int32, device="cuda")
        zk.fixed_base_g1(dk, n, dpts)
        # spot-check fixed-base outputs against the oracle
        words = host_words(dpts).reshape(-1, 16)
        for j in (0, n // 2, n - 1):
            assert words_to_g1_points(words[j])[0] == bn.g1_mul(bn.G1_GEN, ks[j])
        got = zk.msm_g1(dpts, ints_to_dev(sc), n)
        assert got == bn.g1_mul(bn.G1_GEN, sum(a * b for a, b in zip(ks, sc)) % bn.R)


@pytest.mark.parametrize("log_n", [16, 20])
def test_msm_g1_dlog_identity_large(zk, log_n):
    n = (1 << log_n) - 3  # ragged
    ks = synth.fr_limbs(log_n, synth.STREAM_MSM_BASES, n)
    sc = synth.fr_limbs(log_n, synth.STREAM_MSM_SCALARS, n)
    dk, ds = dev_words(ks), dev_words(sc)
    dpts = torch.zeros((n * 16,), dtype=torch.int32, device="cuda")
    zk.fixed_base_g1(dk, n, dpts)
    got = zk.msm_g1(dpts, ds, n)
    k_int, s_int = synth.limbs_to_ints(ks), synth.limbs_to_ints(sc)
    want = bn.g1_mul(bn.G1_GEN, sum(a * b for a, b in zip(k_int, s_int)) % bn.R)
    assert got == want


def test_msm_g1_int8_scalars_large(zk):
    n = 163840
    ks = synth.fr_limbs(9, synth.STREAM_MSM_BASES, n)
    vals = synth.int8_matrix(9, synth.STREAM_MSM_SCALARS, 1, n)[0].astype(int).tolist()
    dk = dev_words(ks)
    dpts = torch.zeros((n * 16,), dtype=torch.int32, device="cuda")
    zk.fixed_base_g1(dk, n, dpts)
    got = zk.msm_g1(dpts, ints_to_dev([v % bn.R for v in vals]), n)
    k_int = synth.limbs_to_ints(ks)
    assert got == bn.g1_mul(bn.G1_GEN, sum(a * b for a, b in zip(k_int, vals)) % bn.R)


def test_msm_g2_small_and_dlog(zk):
    rng = random.Random(5)
    q = bn.G2_GEN
    pts = [bn.g2_mul(q, rng.randrange(1, bn.R)) for _ in range(6)]
    sc = [rng.randrange(bn.R) for _ in range(6)]
    pts2 = pts + [pts[0], None, bn.g2_neg(pts[1])]
    sc2 = sc + [sc[0], 11, sc[1]]
    got = zk.msm_g2(dev_words(g2_points_to_words(pts2)), ints_to_dev(sc2), len(pts2))
    assert got == bn.g2_msm(pts2, sc2)
    n = 5000
    ks = synth.fr_limbs(11, synth.STREAM_MSM_BASES, n)
    vals = synth.int8_matrix(11, synth.STREAM_MSM_SCALARS, 1, n)[0].astype(int).tolist()
    dpts = torch.zeros((n * 32,), dtype=torch.int32, device="cuda")
    zk.fixed_base_g2(dev_words(ks), n, dpts)
    words = host_words(dpts).reshape(-1, 32)
    k_int = synth.limbs_to_ints(ks)
    assert words_to_g2_points(words[17])[0] == bn.g2_mul(q, k_int[17])
    got = zk.msm_g2(dpts, ints_to_dev([v % bn.R for v in vals]), n)
    assert got == bn.g2_mul(q, sum(a * b for a, b in zip(k_int, vals)) % bn.R)


@pytest.mark.parametrize("small", [False, True])
def test_msm_few_distinct_bases(zk, small):
    """Bases cycling over three multiples of G: the buckets, their partial sums
    and the reduction meet equal and opposite points (the doubling and
    cancellation branches of every addition, and sums that pass through
    infinity); checked by the discrete-log identity.  Small signed scalars
    put everything in one window of few, crowded buckets (the quad paths)."""
    rng = random.Random(77 + small)
    n = (1 << 14) + 5
    kk = [rng.randrange(1, bn.R) for _ in range(3)]
    ks = [kk[i % 3] for i in range(n)]
    if small:
        sc = [rng.randrange(-300, 301) for _ in range(n)]
    else:
        sc = [rng.randrange(bn.R) for _ in range(n)]
    dpts = torch.zeros((n * 16,), dtype=torch.int32, device="cuda")
    zk.fixed_base_g1(ints_to_dev(ks), n, dpts)
    got = zk.msm_g1(dpts, ints_to_dev([v % bn.R for v in sc]), n)
    assert got == bn.g1_mul(bn.G1_GEN, sum(a * b for a, b in zip(ks, sc)) % bn.R)
    m = 3000
    dq = torch.zeros((m * 32,), dtype=torch.int32, device="cuda")
    zk.fixed_base_g2(ints_to_dev(ks[:m]), m, dq)
    got2 = zk.msm_g2(dq, ints_to_dev([v % bn.R for v in sc[:m]]), m)
    assert got2 == bn.g2_mul(bn.G2_GEN, sum(a * b for a, b in zip(ks[:m], sc[:m])) % bn.R)


def test_msm_rejects_bad_arguments(zk):
    """Rejections decided before any device memory is touched."""
    d = dev_words(np.zeros((4, 16), dtype=np.uint32))
    with pytest.raises(zk.ZkvcError) as e:
        zk.msm_g1(d, 0, 4)
    assert e.value.code == zk.EINVAL
    with pytest.raises(zk.ZkvcError):
        zk.msm_g2(0, d, 2)
    with pytest.raises(zk.ZkvcError):
        zk.msm_g1(d, d, 2, flags=8)


def test_profile_records_launches_and_selects_one_kernel(zk):
    """The event profiler: every instrumented launch, or only the selected kernel's."""
    log_n = 12
    d = dev_words(synth.fr_limbs(3, synth.STREAM_NTT, 1 << log_n))
    zk.profile_select(None)
    zk.profile_begin()
    zk.ntt_fr(d, log_n, zk.LAYOUT_MONT)
    st = zk.profile_read()
    assert "ntt_pass" in st and st["ntt_pass"][0] >= 2 and st["ntt_pass"][1] > 0
    # butterflies: (N/2) log N over all passes
    assert st["ntt_pass"][2] == (1 << (log_n - 1)) * log_n
    zk.profile_select("no_such_kernel")
    zk.profile_begin()
    zk.ntt_fr(d, log_n, zk.LAYOUT_MONT)
    assert zk.profile_read() == {}
    zk.profile_select("ntt_pass")
    zk.profile_begin()
    zk.ntt_fr(d, log_n, zk.LAYOUT_MONT)
    assert set(zk.profile_read()) == {"ntt_pass"}
    zk.profile_select(["msm_acc_points_g1", "ntt_pass"])
    zk.profile_begin()
    zk.ntt_fr(d, log_n, zk.LAYOUT_MONT)
    assert set(zk.profile_read()) == {"ntt_pass"}
    zk.profile_select(None)
    with pytest.raises(zk.ZkvcError):
        zk.profile_select("x" * 5000)
