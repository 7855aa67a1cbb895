"""Oracle parity at the sizes and in the launch configurations the benchmark reports.

* The batch of 64 mixed-shape CRPC+PSQ proofs (nine shape classes, QAP domains
  2^13..2^16), proved by one zkvc_prove_batch call with the built-in rules and
  again after the autotuner has picked MSM windows, task sizes and NTT pass
  sizes for those domains: every proof against the oracle's closed-form
  trapdoor proof.
* Served proving over the ten classes (the nine plus [49,320] x [320,512]),
  jobs arriving in bursts so that batches mix classes: every proof against the
  trapdoor proof.
* Standalone MSMs with uniform scalars: G2 at 2^16 and 2^20, G1 at 2^24, on the
  very inputs the benchmark times (bases [k_i]G from the fixed-base kernel),
  against the discrete-log identity sum s_i [k_i]G = [sum s_i k_i mod r]G.
* The forward NTT at 2^24 in the internal layout (as timed): the Freivalds
  identity against the input, then plain and coset round trips.

Bar: bit-exact (every result is unique).
"""
import os
import time

import numpy as np
import pytest

import synth
from oracle import bn254 as bn
from oracle import groth16, ntt as ontt, r1cs
from tests.gpu_util import dev_words, host_words

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

WORKERS = max(1, min(16, len(os.sched_getaffinity(0))))
SEED = 0


@pytest.fixture(scope="module")
def zk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_12217_amd import zkvc
    zkvc.lib()
    return zkvc


def _log(msg):
    print(f"[bench-parity] {msg}", flush=True)


_JOBS = {}


def _trapdoor(k):
    shape, X, W, r, s, tox, z = _JOBS["jobs"][k]
    proof, Y = groth16.expected_proof_trapdoor(r1cs.Shape(*shape), r1cs.CRPC_PSQ, tox, X.astype(int).tolist(),
                                                W.astype(int).tolist(), r, s, z)
    return tuple(proof), Y


def _expected_all(jobs, tox, z):
    """Trapdoor proofs of every job, spread over host processes."""
    _JOBS["jobs"] = [(sh, X, W, r, s, tox, z) for sh, X, W, r, s in jobs]
    try:
        if WORKERS > 1 and len(jobs) > 1:
            import multiprocessing as mp
            with mp.get_context("fork").Pool(min(WORKERS, len(jobs))) as pool:
                return pool.map(_trapdoor, range(len(jobs)))
        return [_trapdoor(k) for k in range(len(jobs))]
    finally:
        _JOBS.clear()


def _tune_snapshot(zk):
    return zk.tune_export()


def _tune_restore(zk, text):
    keys = ["msm_g1", "msm_g2", "msm_kdiv", "ntt"]
    zk.tune_import("".join(f"{k} {lg} 0\n" for k in keys for lg in range(0, 34) if not (k == "ntt" and lg > 28)
                           and not (k in ("msm_g1", "msm_g2") and lg > 32)))
    if text.strip():
        zk.tune_import(text)


def test_batch_of_64_bench_mix_built_in_rules_and_tuned(zk):
    jobs = synth.batch_jobs(SEED, 64)
    classes = sorted(set(sh for sh, *_ in jobs))
    assert len(classes) == 9, classes
    tox = synth.toxic_waste(SEED)
    z = synth.crpc_point(SEED)
    keys = {sh: zk.setup(*sh, zk.CRPC_PSQ, tox, z) for sh in classes}
    assert sorted(set(keys[sh].info().log_n for sh in classes)) == [13, 14, 15, 16]
    batch = [(keys[sh], X, W, r, s) for sh, X, W, r, s in jobs]
    t = time.time()
    want = _expected_all(jobs, groth16.Toxic(*tox), z)
    _log(f"64 trapdoor proofs {time.time() - t:.1f}s")
    saved = _tune_snapshot(zk)
    try:
        for tuned in (False, True):
            if tuned:
                nset = zk.autotune(zk.TUNE_MSM_G1 | zk.TUNE_MSM_G2 | zk.TUNE_NTT, 12, 16)
                _log(f"autotune chose {nset} settings")
            got = zk.prove_batch(batch)
            for k, ((sh, X, W, r, s), (Y, proof)) in enumerate(zip(jobs, got)):
                proof_w, Y_w = want[k]
                assert Y.tolist() == Y_w, (tuned, k, sh)
                assert zk.proof_to_tuple(proof) == proof_w, (tuned, k, sh)
        # a sample against the single proof and the library's verifier
        for k in (0, 17, 63):
            sh, X, W, r, s = jobs[k]
            Y1, p1 = zk.prove(keys[sh], X, W, r, s)
            assert zk.proof_to_tuple(p1) == want[k][0]
            assert zk.verify(keys[sh].vk, X, Y1, p1) == 1
    finally:
        _tune_restore(zk, saved)
        for pk in keys.values():
            pk.close()


def test_served_ten_classes_with_paper_shape(zk):
    classes = synth.served_classes()
    assert len(classes) == 10 and classes[-1] == synth.PAPER_SHAPE
    tox = synth.toxic_waste(SEED)
    z = synth.crpc_point(SEED)
    keys = {sh: zk.setup(*sh, zk.CRPC_PSQ, tox, z) for sh in classes}
    # the benchmark's arrival stream at 200 req/s, first 40 jobs, plus two
    # paper-shape jobs in the middle of a burst
    _, jobs = synth.served_jobs(SEED, 200, 40)
    extra = synth.served_jobs(SEED, 2000, 60)[1]
    jobs += [j for j in extra if j[0] == synth.PAPER_SHAPE][:2]
    assert set(sh for sh, *_ in jobs) == set(classes)
    t = time.time()
    want = _expected_all(jobs, groth16.Toxic(*tox), z)
    _log(f"{len(jobs)} trapdoor proofs {time.time() - t:.1f}s")
    srv = zk.Server(max_batch=64)
    try:
        # three bursts: the jobs of a burst are queued while the previous one proves
        tickets = []
        for lo, hi in ((0, 10), (10, 30), (30, len(jobs))):
            tickets += [srv.submit(keys[sh], X, W, r, s) for sh, X, W, r, s in jobs[lo:hi]]
        results = [srv.wait(tk) for tk in tickets]
    finally:
        srv.close()
    sizes = []
    for k, ((sh, X, W, r, s), (Y, proof, res)) in enumerate(zip(jobs, results)):
        assert res.status == zk.OK
        sizes.append(res.batch_size)
        assert Y.tolist() == want[k][1], (k, sh)
        assert zk.proof_to_tuple(proof) == want[k][0], (k, sh)
    assert max(sizes) > 1
    for pk in keys.values():
        pk.close()


def _dot_mod_r(k_limbs, s_limbs):
    """sum_i k_i s_i mod r over [n, 8] limb arrays (chunked to bound memory)."""
    acc = 0
    step = 1 << 20
    for lo in range(0, k_limbs.shape[0], step):
        ks = synth.limbs_to_ints(k_limbs[lo:lo + step])
        ss = synth.limbs_to_ints(s_limbs[lo:lo + step])
        acc = (acc + sum(a * b for a, b in zip(ks, ss))) % bn.R
    return acc


@pytest.mark.parametrize("group,log_n", [(2, 16), (2, 20), (1, 24)])
def test_uniform_msm_at_benchmark_sizes(zk, group, log_n):
    n = 1 << log_n
    ks = synth.fr_limbs(SEED, synth.STREAM_MSM_BASES, n)
    sc = synth.fr_limbs(SEED, synth.STREAM_MSM_SCALARS, n)
    _log(f"G{group} MSM 2^{log_n}")
    dk = dev_words(ks)
    ds = dev_words(sc)
    pts = torch.zeros((n * (16 if group == 1 else 32),), dtype=torch.int32, device="cuda")
    (zk.fixed_base_g1 if group == 1 else zk.fixed_base_g2)(dk, n, pts)
    del dk
    got = (zk.msm_g1 if group == 1 else zk.msm_g2)(pts, ds, n)
    del pts, ds
    torch.cuda.empty_cache()
    t = time.time()
    e = _dot_mod_r(ks, sc)
    want = bn.g1_mul(bn.G1_GEN, e) if group == 1 else bn.g2_mul(bn.G2_GEN, e)
    _log(f"dlog sum {time.time() - t:.1f}s")
    assert got == want


def test_ntt_forward_2_24_internal_layout(zk):
    log_n = 24
    n = 1 << log_n
    x = synth.fr_limbs(SEED, synth.STREAM_NTT, n)
    d = dev_words(x)
    m = torch.zeros_like(d)
    zk.field_op(zk.FR, zk.OP_TO_MONT, d, None, m, n)
    zk.ntt_fr(m, log_n, zk.LAYOUT_MONT)       # the transform the benchmark times
    zk.field_op(zk.FR, zk.OP_FROM_MONT, m, None, d, n)
    X = host_words(d).reshape(-1, 8)
    del m
    t = time.time()
    ok = ontt.freivalds_check_parallel(synth.limbs_to_ints(x), synth.limbs_to_ints(X),
                                       0x1234567890ABCDEF1234567890ABCDEF, WORKERS)
    _log(f"Freivalds 2^24 {time.time() - t:.1f}s")
    assert ok
    # canonical-layout round trips through the inverse and the coset pair
    zk.ntt_fr(d, log_n, zk.NTT_INVERSE)
    assert np.array_equal(host_words(d).reshape(-1, 8), x)
    zk.ntt_fr(d, log_n, zk.NTT_COSET)
    zk.ntt_fr(d, log_n, zk.NTT_COSET | zk.NTT_INVERSE)
    assert np.array_equal(host_words(d).reshape(-1, 8), x)
