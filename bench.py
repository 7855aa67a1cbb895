#!/usr/bin/env python3
"""Throughput of the Groth16 matmul prover on one MI355X.

Workload (the paper's headline shape, Section I / Section IV): prove Y = X W
for X [49, 320] and W [320, 512] with int8 entries drawn uniformly from
[-128, 127] (seeded; they stand in for quantized ViT activations and weights),
over BN254, with the proving key resident in device memory.

  step   = one complete proof with zkVC's circuit (CRPC + PSQ, QAP domain 2^16):
           witness and evaluation vectors, QAP quotient (3 iNTT, 3 coset NTT,
           pointwise: h on the coset), G1 MSMs (A, B1, L, H), G2 MSM (B),
           assembly.  X and W are resident in device memory when the timed
           region starts and Y is written there (zkvc_prove_device); the
           256-byte proof comes back to the host.
  value  = CRPC + PSQ proofs per second.
Timed beside it in the same run: the same proofs from host buffers (PCIe
included) and by graph replay, the plain per-product circuit of the same
matmul (8,028,160 constraints, domain 2^23), standalone G1 and G2 MSMs and Fr
NTTs, a batch of 64 mixed-shape proofs, served proving at several arrival
rates, Table II's four rows, the Spartan backend, the integer-VALU peak, and
the CPU oracle on one whole proof.

Prints one JSON line.  Only one GPU is supported (--gpus 1).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402

METRIC = "matmul Groth16 proofs/s + MSM Mpts/s (1 GPU); p50/p99 proof latency served"
SHAPE = (49, 320, 512)
PEAK_MAD = 256 * 64 * 2.4e9          # u32 multiply-adds per second (full-rate v_mad_u64_u32)
MAD_PER_FMUL = 136                   # 8-limb Montgomery product: 64 product + 72 reduction MADs
FMUL_PER_UNIT = {                    # algorithmic Fq/Fr multiplications per counted unit
    "msm_acc_points_g1": 10,         # G1 mixed addition (8M + 2S)
    "msm_acc_points_g2": 30,         # G2 mixed addition over Fq2
    "msm_bitplanes_g1": 14,          # G1 general addition (12M + 2S)
    "msm_bitplanes_g2": 42,
    "msm_gridsums_g1": 14,           # G1 general additions of the grid reduction's row and column sums
    "msm_gridsums_g2": 42,
    "ntt_pass": 1,                   # radix-2 butterfly
}


# Measured HBM traffic per launch of a kernel (from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE runs,
# scaled by the same counters on a device copy of known size) is recorded in profiles/ with a fingerprint
# of the sources the kernel is built from; it is reported only while the sources still match.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_per_launch.md")
KERNEL_SOURCES = ["paper_2504_12217_amd/csrc/msm.hip", "paper_2504_12217_amd/csrc/curve.hpp",
                  "paper_2504_12217_amd/csrc/field.hpp", "paper_2504_12217_amd/csrc/ntt.hip"]


def source_fingerprint():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def recorded_traffic(kernel, workload):
    """Bytes per launch recorded for (kernel, workload), or None if absent or the sources changed."""
    try:
        lines = open(TRAFFIC_FILE).read().splitlines()
    except OSError:
        return None
    fp = source_fingerprint()
    for ln in lines:
        # | kernel | workload | fingerprint | fetch bytes/launch | write bytes/launch | total |
        cells = [c.strip().strip("`") for c in ln.strip().strip("|").split("|")]
        if len(cells) >= 6 and cells[0] == kernel and cells[1] == workload and cells[2] == fp:
            try:
                return float(cells[5])
            except ValueError:
                return None
    return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def roofline(stats, workload=None, measured=None):
    """Roofline entry for the kernel with the most device time (peak: the
    nominal 64 lane-ops per compute unit per clock at 2.4 GHz; beside it the
    fraction of the microbenchmark's measured rate, if given)."""
    modeled = {k: v for k, v in stats.items() if k in FMUL_PER_UNIT} or stats
    if not modeled:
        return None, None
    name, (launches, total_ms, work) = max(modeled.items(), key=lambda kv: kv[1][1])
    avg_ms = total_ms / max(launches, 1)
    per_unit = FMUL_PER_UNIT.get(name)
    if per_unit is None:
        return name, None
    mad_per_launch = work / launches * per_unit * MAD_PER_FMUL
    achieved = mad_per_launch / (avg_ms * 1e-3) / 1e12
    peak = PEAK_MAD / 1e12
    traffic = recorded_traffic(name, workload) if workload else None
    out = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 3),
           "unit": "T u32-MAD/s", "frac": round(achieved / peak, 4),
           "traffic": None if traffic is None else round(traffic),
           "kernel": name, "launches": launches, "avg_launch_ms": round(avg_ms, 4),
           "work_units_per_launch": work / launches,
           "timing": "HIP events bound to each launch on its stream (hipExtLaunchKernel: the kernel's own start and end)"}
    if measured:
        out["measured_peak"] = round(measured / 1e12, 3)
        out["frac_vs_measured_peak"] = round(achieved * 1e12 / measured, 4)
    return name, out


def time_proofs(zk, one, steps, warmup, profile):
    """Times `steps` calls of one() (a proof) after `warmup` ones.  With profile set, the warm-up
    proofs time every instrumented launch (the per-kernel table), a few more
    untimed proofs pick the kernel with an algorithmic work model that takes
    the most device time, and the timed proofs record only that kernel's
    launches (two HIP events per launch), which the roofline reports.
    Returns (seconds, per-proof latencies, timed-region stats, warm-up stats)."""
    import torch
    stats_all = None
    if profile:
        zk.profile_select(None)
        zk.profile_begin()
    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    if profile:
        stats_all = zk.profile_read()
        # the timed proofs record only the kernel with the most device time
        # among the single-kernel scopes with an algorithmic work model
        # (msm_sort, say, spans several kernels), so that the timed region
        # carries two event records per launch of that kernel and no more;
        # a few untimed proofs past the warm-up pick it
        zk.profile_select(sorted(FMUL_PER_UNIT))
        zk.profile_begin()
        for _ in range(max(5, warmup)):
            one()
        torch.cuda.synchronize()
        modeled = zk.profile_read()
        dom = max(modeled, key=lambda k: modeled[k][1]) if modeled else None
        zk.profile_select([dom] if dom else sorted(FMUL_PER_UNIT))
        zk.profile_begin()
    lat = []
    t0 = time.perf_counter()
    for _ in range(steps):
        t = time.perf_counter()
        one()
        lat.append(time.perf_counter() - t)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    stats = None
    if profile:
        stats = zk.profile_read()
        zk.profile_select(None)
    return total, lat, stats, stats_all


FR_ORDER = 21888242871839275222246405745257275088548364400416034343698204186575808495617


def int8_scalar_limbs(seed, n):
    """[n, 8] uint32 limbs of int8 values (uniform in [-128, 127], negatives as r - |v|)."""
    v = synth.int8_matrix(seed, synth.STREAM_MSM_SCALARS, 1, n).reshape(-1).astype(np.int64)
    return synth.ints_to_limbs([int(x) % FR_ORDER for x in v])


def msm_rate(zk, n, seed=0, group=1, int8=False, reps=3):
    """Points per second of the standalone MSM: bases [k_i]G from the fixed-base kernel."""
    import torch
    ks = synth.fr_limbs(seed, synth.STREAM_MSM_BASES, n)
    sc = int8_scalar_limbs(seed, n) if int8 else synth.fr_limbs(seed, synth.STREAM_MSM_SCALARS, n)
    dk = torch.from_numpy(ks.view(np.int32).copy()).cuda()
    ds = torch.from_numpy(sc.view(np.int32).copy()).cuda()
    pts = torch.zeros((n * (16 if group == 1 else 32),), dtype=torch.int32, device="cuda")
    (zk.fixed_base_g1 if group == 1 else zk.fixed_base_g2)(dk, n, pts)
    del dk
    run = zk.msm_g1 if group == 1 else zk.msm_g2
    run(pts, ds, n)  # warm-up (workspace growth)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        run(pts, ds, n)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    del pts, ds
    torch.cuda.empty_cache()
    return n / dt / 1e6, dt * 1e3


def ntt_rate(zk, log_n, seed=0, reps=5):
    """Forward Fr NTT of 2^log_n elements in the internal layout (natural order in and out)."""
    import torch
    n = 1 << log_n
    x = synth.fr_limbs(seed, synth.STREAM_NTT, n)
    d = torch.from_numpy(x.view(np.int32).copy()).cuda()
    zk.ntt_fr(d, log_n, zk.LAYOUT_MONT)
    torch.cuda.synchronize()
    zk.profile_begin()
    t0 = time.perf_counter()
    for _ in range(reps):
        zk.ntt_fr(d, log_n, zk.LAYOUT_MONT)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    st = zk.profile_read()
    del d
    torch.cuda.empty_cache()
    out = {"melem_per_s": round(n / dt / 1e6, 2), "ms": round(dt * 1e3, 4)}
    if "ntt_pass" in st:
        launches, total_ms, work = st["ntt_pass"]
        passes = launches // reps
        # each pass reads and writes every element once: 64 B per element
        gbs = passes * n * 64 / (total_ms / reps * 1e-3) / 1e9
        mad = work / reps * MAD_PER_FMUL / (total_ms / reps * 1e-3) / 1e12
        out.update({"passes": passes, "pass_ms_avg": round(total_ms / launches, 4),
                    "hbm": {"achieved_gb_s": round(gbs, 1), "peak_gb_s": 8000, "frac": round(gbs / 8000, 4)},
                    "alu": {"achieved_t_mad_s": round(mad, 3), "peak": round(PEAK_MAD / 1e12, 3),
                            "frac": round(mad * 1e12 / PEAK_MAD, 4)}})
    return out


def batch_section(zk, seed, count=64, reps=3):
    """Throughput of batched CRPC+PSQ proving over mixed shapes (one key per shape class)."""
    import torch
    jobs = synth.batch_jobs(seed, count)
    tox = synth.toxic_waste(seed)
    z = synth.crpc_point(seed)
    keys = {}
    t0 = time.perf_counter()
    for shape, *_ in jobs:
        if shape not in keys:
            keys[shape] = zk.setup(*shape, zk.CRPC_PSQ, tox, z)
    setup_s = time.perf_counter() - t0
    batch = [(keys[sh], X, W, r, s) for sh, X, W, r, s in jobs]

    def timed():
        zk.prove_batch(batch)  # warm-up (workspace growth)
        torch.cuda.synchronize()
        lat = []
        t0 = time.perf_counter()
        for _ in range(reps):
            t = time.perf_counter()
            res = zk.prove_batch(batch)
            lat.append(time.perf_counter() - t)
        return time.perf_counter() - t0, lat, res

    dt0, _, _ = timed()
    # then with the autotuner's picks for these sizes (MSM window and task size, NTT pass size)
    t0 = time.perf_counter()
    nset = zk.autotune(zk.TUNE_MSM_G1 | zk.TUNE_MSM_G2 | zk.TUNE_NTT, 12, 16)
    tune_s = time.perf_counter() - t0
    dt, lat, outs = timed()
    table = zk.tune_export().split("\n")[:-1]
    # the other sections keep the built-in rules (value 0 restores a rule)
    zk.tune_import("".join(" ".join(line.split()[:2]) + " 0\n" for line in table if line.strip()))
    ok = verify_all(zk, [(keys[sh].vk, X, Y, p) for (sh, X, W, r, s), (Y, p) in zip(jobs, outs)])
    # the same jobs one by one, for comparison
    t0 = time.perf_counter()
    for pk, X, W, r, s in batch:
        zk.prove(pk, X, W, r, s)
    single_s = time.perf_counter() - t0
    for pk in keys.values():
        pk.close()
    classes = sorted(set(sh for sh, *_ in jobs))
    return {"workload": f"{count} CRPC+PSQ proofs, a=49, (n, b) drawn per proof from {{64,128,320}}x{{64,256,512}} "
                        f"({len(classes)} shape classes, QAP domains 2^13..2^16), one zkvc_prove_batch call",
            "proofs_per_s": round(count * reps / dt, 2), "ms_per_batch": round(dt / reps * 1e3, 3),
            "proofs_per_s_builtin_rules": round(count * reps / dt0, 2),
            "autotune": {"seconds": round(tune_s, 2), "settings": nset, "table": table,
                         "note": "applied to this section's tuned run only; the built-in rules are restored after it"},
            "batch_latency_ms_max": round(max(lat) * 1e3, 3),
            "same_jobs_one_by_one_proofs_per_s": round(count / single_s, 2),
            "setup_s_all_keys": round(setup_s, 3), "verified_all": ok}


SERVE_RATES = (5, 20, 50, 100, 200, 2000)  # the last one overloads a one-at-a-time prover


def verify_all(zk, items, threads=16):
    """zkvc_verify on every (vk, X, Y, proof), on host threads (the verifier is
    host code; ctypes releases the interpreter lock during the call)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return all(v == 1 for v in ex.map(lambda it: zk.verify(*it), items))


def serve_section(zk, seed, rates=SERVE_RATES, max_batch=64, seconds=20.0, max_jobs=2000):
    """Poisson arrivals of CRPC+PSQ jobs over 10 shape classes (the batch mix plus the paper shape),
    proved by the library's server; latency = submission to results written.  Each rate runs
    min(max_jobs, rate * seconds) jobs (at least 40)."""
    import torch
    classes = synth.served_classes()
    tox = synth.toxic_waste(seed)
    z = synth.crpc_point(seed)
    keys = {sh: zk.setup(*sh, zk.CRPC_PSQ, tox, z) for sh in classes}
    # warm the server (a server in steady state): every class alone twice in a
    # row (both batch generations size their buffers and factor tables for it),
    # then one batch of all classes together
    srv = zk.Server(max_batch=max_batch)
    for sh in classes:
        for _ in range(2):
            srv.wait(srv.submit(keys[sh], *synth.matmul_inputs(seed, *sh), 3, 5))
    for t in [srv.submit(keys[sh], *synth.matmul_inputs(seed, *sh), 3, 5) for sh in classes]:
        srv.wait(t)
    # and bursts of the largest class, so that the first few batch slots of
    # both generations hold buffers of its size
    big = max(classes, key=lambda sh: sh[1] * sh[2])
    for _ in range(2):
        for t in [srv.submit(keys[big], *synth.matmul_inputs(seed, *big), 3, 5) for _ in range(8)]:
            srv.wait(t)
    # and full bursts of every class in turn, so that batches as large as
    # the highest rate forms (tens of mixed jobs) find their buffers sized
    for _ in range(2):
        burst = [classes[q % len(classes)] for q in range(max_batch)]
        for t in [srv.submit(keys[sh], *synth.matmul_inputs(seed, *sh), 3, 5) for sh in burst]:
            srv.wait(t)
    out = {}
    all_ok = True
    for lam in rates:
        count = int(max(40, min(max_jobs, lam * seconds)))
        gaps, jobs = synth.served_jobs(seed, lam, count)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        due = t0
        tickets = []
        for j, (sh, X, W, r, s) in enumerate(jobs):
            due += gaps[j]
            pause = due - time.perf_counter()
            if pause > 0:
                time.sleep(pause)
            tickets.append(srv.submit(keys[sh], X, W, r, s))
        got = [srv.wait(t) for t in tickets]
        span = time.perf_counter() - t0
        res = [g[2] for g in got]
        ok = verify_all(zk, [(keys[sh].vk, X, g[0], g[1]) for (sh, X, W, r, s), g in zip(jobs, got)])
        all_ok = all_ok and ok
        lat = sorted(r.latency_ms for r in res)
        out[f"{lam}_req_s"] = {"jobs": count, "seconds": round(span, 2), "proofs_per_s": round(count / span, 2),
                               "p50_ms": round(lat[len(lat) // 2], 3),
                               "p99_ms": round(lat[min(len(lat) - 1, int(0.99 * len(lat)))], 3),
                               "mean_batch": round(sum(r.batch_size for r in res) / count, 2),
                               "max_batch": max(r.batch_size for r in res), "verified_all": ok}
        log(f"served {lam} req/s: {count} jobs, p50 {out[f'{lam}_req_s']['p50_ms']} ms, "
            f"p99 {out[f'{lam}_req_s']['p99_ms']} ms")
    srv.close()
    for pk in keys.values():
        pk.close()
    return {"workload": "Poisson arrivals of CRPC+PSQ proof jobs, shapes uniform over 10 classes: a=49, (n, b) in "
                        "{64,128,320}x{64,256,512} and (320, 512); keys resident in HBM; one server, continuous "
                        f"batching (max {max_batch} per batch); latency = submission to proof on the host; each "
                        f"rate runs min({max_jobs}, {seconds:g} s x rate) jobs, at least 40",
            "rates": out, "verified_all": all_ok}


def spartan_section(zk, seed, steps=10, warmup=2):
    """The Spartan backend (zkVC-S) on the GPU: CRPC+PSQ and CRPC at the paper shape and the
    Table II shape.  The commitment generators are [k_j]G for seeded k_j (their discrete logarithms
    are known, which serves measurement only: the cost does not depend on the generators)."""
    import torch
    out = {}
    z = synth.crpc_point(seed)
    for sh in ((49, 320, 512), (49, 64, 128)):
        for name in ("CRPC_PSQ", "CRPC"):
            kind = getattr(zk, name)
            info = zk.spartan_info(*sh, kind)
            ks = synth.fr_limbs(seed + 17, synth.STREAM_MSM_BASES, info.cols)
            dk = torch.from_numpy(ks.view(np.int32).copy()).cuda()
            pts = torch.zeros((info.cols * 16,), dtype=torch.int32, device="cuda")
            zk.fixed_base_g1(dk, info.cols, pts)
            words = pts.cpu().numpy().view(np.uint32).reshape(-1, 16)
            ints = synth.limbs_to_ints(words.reshape(-1, 8))
            gens = [(ints[2 * i], ints[2 * i + 1]) for i in range(info.cols)]
            log(f"Spartan {name} {sh}")
            key = zk.SpartanKey(*sh, kind, z, gens)
            X, W = synth.matmul_inputs(seed, *sh)
            for _ in range(warmup):
                key.prove(X, W)
            lat = []
            t0 = time.perf_counter()
            for _ in range(steps):
                t = time.perf_counter()
                Y, proof = key.prove(X, W)
                lat.append(time.perf_counter() - t)
            dt = (time.perf_counter() - t0) / steps
            tv = time.perf_counter()
            ok = key.verify(X, Y, proof) == 1
            verify_ms = (time.perf_counter() - tv) * 1e3
            key.close()
            lat.sort()
            out[f"{name}_{sh[0]}x{sh[1]}x{sh[2]}"] = {
                "ms_per_proof": round(dt * 1e3, 3), "proofs_per_s": round(1 / dt, 2),
                "p50_ms": round(lat[len(lat) // 2] * 1e3, 3), "verify_ms_host": round(verify_ms, 2),
                "proof_bytes": int(info.proof_bytes), "sumcheck_vars": [int(info.sx), int(info.sy)],
                "commitment_rows_x_cols": [int(info.rows), int(info.cols)], "verified": ok}
    out["paper_context"] = {"note": "Table II Spartan prove / verify on a 16-core Threadripper PRO 3955WX (CPU, "
                                    "other hardware; shape inferred as [49,64]x[64,128])",
                            "CRPC_PSQ_s": [1.75, 0.05], "CRPC_s": [1.79, 0.08]}
    return out


TABLE2_KINDS = (("PLAIN_ADD", "no CRPC, no PSQ"), ("PLAIN_PSQ", "no CRPC, PSQ"), ("CRPC", "CRPC, no PSQ"),
                ("CRPC_PSQ", "CRPC, PSQ"))


def table2_section(zk, seed, shapes=((49, 64, 128), (49, 320, 512)), steps=5):
    """The four rows of the paper's Table II ablation (groth16 columns) proved on the GPU."""
    X0 = {}
    out = {}
    tox = synth.toxic_waste(seed)
    z = synth.crpc_point(seed)
    r, s = synth.prover_randomness(seed)
    for sh in shapes:
        X, W = synth.matmul_inputs(seed, *sh)
        X0[sh] = (X, W)
        row = {}
        for name, label in TABLE2_KINDS:
            kind = getattr(zk, name)
            log(f"Table II {name} {sh}")
            pk = zk.setup(*sh, kind, tox, z if name.startswith("CRPC") else None)
            info = pk.info()
            for _ in range(3):  # first calls on a new key size its workspaces
                t0 = time.perf_counter()
                zk.prove(pk, X, W, r, s)
            n = max(steps, min(50, int(0.05 / (time.perf_counter() - t0))))
            t0 = time.perf_counter()
            for _ in range(n):
                Y, proof = zk.prove(pk, X, W, r, s)
            dt = (time.perf_counter() - t0) / n
            ok = zk.verify(pk.vk, X, Y, proof) == 1
            row[name] = {"ablation_row": label, "ms_per_proof": round(dt * 1e3, 3), "proofs_timed": n,
                         "proofs_per_s": round(1 / dt, 2), "qap_domain_log2": info.log_n,
                         "a_query": info.a_query, "l_query": info.l_query, "verified": ok}
            pk.close()
        out[f"{sh[0]}x{sh[1]}x{sh[2]}"] = row
    out["paper_context"] = {"note": "Table II groth16 prove times on a 16-core Threadripper PRO 3955WX (CPU, other "
                                    "hardware; shape of the microbenchmark inferred as [49,64]x[64,128])",
                            "PLAIN_ADD_s": 9.12, "PLAIN_PSQ_s": 8.69, "CRPC_s": 1.01, "CRPC_PSQ_s": 0.73}
    return out


_CPU = {}


def _cpu_msm_part(job):
    """One chunk of a multi-scalar sum by the oracle's double-and-add (bases cycled)."""
    from oracle import bn254 as bn
    name, group, lo, hi = job
    sc = _CPU[name][lo:hi]
    bases = _CPU["bases1"] if group == 1 else _CPU["bases2"]
    pts = [bases[k % len(bases)] for k in range(lo, hi)]
    return (bn.g1_msm if group == 1 else bn.g2_msm)(pts, sc)


def _cpu_quotient(_):
    from oracle import qap
    return qap.quotient_coset(_CPU["aev"], _CPU["bev"], _CPU["cev"])


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(X, W, tox, z, r, s, workers=None, chunk=2048):
    """The oracle prover, unmodified, for one CRPC + PSQ proof of the paper shape
    on every host core: witness and evaluation vectors, the QAP quotient (seven
    transforms of 2^16 by the oracle's recursive FFT, in one process), and the
    five multi-scalar sums A, B1, B2, L, H over all their terms by the oracle's
    double-and-add, split into chunks over a process pool and the chunk sums
    added, then the assembly's scalar multiplications.  Nothing is sampled.
    The proving key's bases are stood in for by 8 fixed points cycled (the
    cost of double-and-add does not depend on the base), which saves the
    oracle's key generation (about an hour of Python)."""
    import multiprocessing as mp
    import platform
    from oracle import bn254 as bn
    from oracle import r1cs
    workers = workers or len(os.sched_getaffinity(0))
    sh = r1cs.Shape(*synth.PAPER_SHAPE)
    kind = r1cs.CRPC_PSQ
    Xl, Wl = X.astype(int).tolist(), W.astype(int).tolist()
    t_start = time.perf_counter()
    a, _ = r1cs.assignment(sh, kind, Xl, Wl, z)
    aev, bev, cev = r1cs.eval_vectors(sh, kind, a, z)
    t_wit = time.perf_counter() - t_start
    ell = r1cs.num_public(sh)
    w0 = r1cs.first_witness(sh)
    _CPU.update({"A": a[:ell + 1], "BW": a[w0:w0 + sh.n * sh.b], "L": a[w0:], "aev": aev, "bev": bev, "cev": cev,
                 "bases1": [bn.g1_mul(bn.G1_GEN, 1000 + k) for k in range(8)],
                 "bases2": [bn.g2_mul(bn.G2_GEN, 1000 + k) for k in range(8)]})
    parts = {}
    try:
        with mp.get_context("fork").Pool(workers) as pool:
            hq = pool.map_async(_cpu_quotient, [0])
            jobs = []
            for name, key, group in (("A", "A", 1), ("B1", "BW", 1), ("B2", "BW", 2), ("L", "L", 1)):
                n = len(_CPU[key])
                jobs += [((name, key, group), lo, min(n, lo + chunk)) for lo in range(0, n, chunk)]
            res = pool.map_async(_cpu_msm_part, [(key, g, lo, hi) for (nm, key, g), lo, hi in jobs])
            h = hq.get()[0]
            t_qap = time.perf_counter() - t_start - t_wit
            _CPU["H"] = h
            hjobs = [("H", "H", 1, lo, min(len(h), lo + chunk)) for lo in range(0, len(h), chunk)]
            # the H chunks see the quotient: a second pool forked after it exists
            with mp.get_context("fork").Pool(workers) as pool2:
                hres = pool2.map(_cpu_msm_part, [(key, g, lo, hi) for nm, key, g, lo, hi in hjobs])
            for ((nm, key, g), lo, hi), v in zip(jobs, res.get()):
                parts.setdefault(nm, []).append(v)
            parts["H"] = hres
    finally:
        _CPU.clear()
    sums = {nm: None for nm in parts}
    for nm, vs in parts.items():
        add = bn.g2_add if nm == "B2" else bn.g1_add
        for v in vs:
            sums[nm] = add(sums[nm], v)
    # assembly: A + r delta1, B + s delta2, B1 + s delta1, C = L + H + s A + r B1 - r s delta1
    d1, d2 = bn.g1_mul(bn.G1_GEN, 7), bn.g2_mul(bn.G2_GEN, 7)
    A = bn.g1_add(sums["A"], bn.g1_mul(d1, r))
    bn.g2_add(sums["B2"], bn.g2_mul(d2, s))
    B1 = bn.g1_add(sums["B1"], bn.g1_mul(d1, s))
    C = bn.g1_add(bn.g1_add(sums["L"], sums["H"]), bn.g1_add(bn.g1_mul(A, s), bn.g1_mul(B1, r)))
    bn.g1_add(C, bn.g1_neg(bn.g1_mul(d1, r * s % bn.R)))
    total = time.perf_counter() - t_start
    nterms = {nm: sum(1 for _ in vs) for nm, vs in parts.items()}
    return {"value": round(1.0 / total, 6), "unit": "proofs/s", "cores": workers, "kind": "oracle",
            "sample": (f"one whole CRPC+PSQ proof of [49,320]x[320,512], nothing sampled: witness and evaluation "
                       f"vectors ({t_wit:.1f} s, one process), QAP quotient (7 transforms of 2^16, one process, "
                       f"{t_qap:.1f} s) overlapped with the A, B1, B2, L multi-scalar sums, then the H sum; all "
                       f"five sums by double-and-add over every term, in chunks of {chunk} on a pool of {workers} "
                       f"processes; bases cycled over 8 fixed points"),
            "seconds_per_proof": round(total, 2), "cpu_model": cpu_model(),
            "python": platform.python_version(), "msm_chunks": nterms}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--circuit", choices=("crpc_psq", "plain"), default="crpc_psq",
                    help="circuit of the timed step (the other one is timed beside it unless --no-plain)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-msm", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-table2", action="store_true")
    ap.add_argument("--no-spartan", action="store_true")
    ap.add_argument("--no-valu-peak", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=20.0,
                    help="arrivals per served rate: min(--serve-max-jobs, rate x this), at least 40")
    ap.add_argument("--serve-max-jobs", type=int, default=2000)
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="first copy this many MiB device to device (a known-size kernel for counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the prover runs on a single MI355X "
              "(multi-GPU sharding is described, not implemented); run with --gpus 1", file=sys.stderr)
        return 2
    import torch
    from paper_2504_12217_amd import zkvc
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    zkvc.lib()
    if args.calib_copy_mb:
        nb = args.calib_copy_mb << 20
        src = torch.ones(nb // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy of {args.calib_copy_mb} MiB done")
        del src, dst
    valu = None
    if not args.no_valu_peak:
        log("integer-VALU peak microbenchmark (v_mad_u64_u32)")
        valu = zkvc.valu_peak()
    a, n, b = SHAPE
    seed = args.seed
    X, W = synth.matmul_inputs(seed, a, n, b)
    tox = synth.toxic_waste(seed)
    z = synth.crpc_point(seed)
    r, s = synth.prover_randomness(seed)

    main_kind = zkvc.CRPC_PSQ if args.circuit == "crpc_psq" else zkvc.PLAIN
    log(f"setup {args.circuit}")
    t0 = time.perf_counter()
    pk = zkvc.setup(a, n, b, main_kind, tox, z if main_kind == zkvc.CRPC_PSQ else None)
    setup_crpc_s = time.perf_counter() - t0
    # X and W resident in HBM, Y written there: nothing but the proof crosses PCIe
    Xd = torch.from_numpy(X).to("cuda")
    Wd = torch.from_numpy(W).to("cuda")
    Yd = torch.empty((a, b), dtype=torch.int32, device="cuda")
    prove_dev = lambda: zkvc.prove_device(pk, Xd, Wd, r, s, Yd)  # noqa: E731
    log(f"timing {args.steps} {args.circuit} proofs (operands in HBM)")
    total, lat, stats, stats_warm = time_proofs(zkvc, prove_dev, args.steps, args.warmup, profile=True)
    st = pk.last_stats()
    proof = prove_dev()
    Y = Yd.cpu().numpy()
    Yh, proof_h = zkvc.prove(pk, X, W, r, s)
    ok = zkvc.verify(pk.vk, X, Y, proof) == 1 and bytes(proof_h) == bytes(proof) and np.array_equal(Yh, Y)
    # the host-buffer interface: X, W cross PCIe in the call and Y comes back
    steps_e = max(5, args.steps // 3)
    log(f"timing {steps_e} {args.circuit} proofs from host buffers")
    th, _, _, _ = time_proofs(zkvc, lambda: zkvc.prove(pk, X, W, r, s), steps_e, 2, profile=False)
    # the same proofs replaying a captured HIP graph instead of eager launches
    log(f"timing {steps_e} {args.circuit} proofs with graph replay")
    prev_graphs = zkvc.set_graphs(1)
    te, late, _, _ = time_proofs(zkvc, prove_dev, steps_e, 2, profile=False)
    zkvc.set_graphs(prev_graphs)
    stage_ms = {"witness": round(st.witness_ms, 3), "qap_ntt": round(st.ntt_ms, 3),
                "msm_all_concurrent": round(st.msm_ms, 3), "host_windows_and_assembly": round(st.host_ms, 3),
                "total_wall": round(st.total_ms, 3)}
    pk.close()
    mpeak = valu["mad_per_s"] if valu else None
    dom_name, roof = roofline(stats, "crpc_psq_49x320x512" if main_kind == zkvc.CRPC_PSQ else "plain_49x320x512",
                              mpeak)
    lat_ms = sorted(x * 1e3 for x in lat)
    ms_per_step = total / args.steps * 1e3
    out = {
        "metric": METRIC,
        "value": round(args.steps / total, 3),
        "unit": "proofs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "Groth16/BN254 proof of Y=XW, X[49,320] int8, W[320,512] int8, " + (
                   "CRPC+PSQ circuit (320 constraints, QAP domain 2^16)" if main_kind == zkvc.CRPC_PSQ else
                   "plain per-product circuit (8,028,160 constraints, QAP domain 2^23)") + ", proving key in HBM",
                   "global_batch": 1, "seq_len": None, "parallelism": "none (1 GPU)", "seed": seed},
        "verified": ok,
        "latency_ms": {"p50": round(lat_ms[len(lat_ms) // 2], 3),
                       "p99": round(lat_ms[min(len(lat_ms) - 1, int(0.99 * len(lat_ms)))], 3)},
        "stage_ms_last_proof": stage_ms,
        "host_buffers": {"proofs_per_s": round(steps_e / th, 3), "ms_per_proof": round(th / steps_e * 1e3, 3),
                         "note": "zkvc_prove with X, W and Y in host memory (PCIe-inclusive: ~276 KB cross "
                                 "per proof); value above uses zkvc_prove_device with operands in HBM"},
        "graph_replay": {"proofs_per_s": round(steps_e / te, 3), "ms_per_proof": round(te / steps_e * 1e3, 3),
                         "note": "the same proofs replaying a captured HIP graph (zkvc_set_graphs(1)); "
                                 "value above uses the default eager launches on three streams"},
        "setup_s": round(setup_crpc_s, 3),
        "roofline": roof,
        "valu_peak": None if valu is None else {
            "what": "v_mad_u64_u32 microbenchmark (zkvc_valu_peak): 8 blocks of 256 threads per CU, 16 "
                    "independent multiply-add chains per thread",
            "t_mad_per_s": round(valu["mad_per_s"] / 1e12, 3), "clock_ghz": round(valu["clock_ghz"], 3),
            "lane_ops_per_cu_clk": round(valu["lane_ops_per_cu_clk"], 2), "compute_units": valu["compute_units"],
            "nominal_t_mad_per_s": round(PEAK_MAD / 1e12, 3)},
        "kernels_warmup": {k: {"launches": v[0], "total_ms": round(v[1], 3)} for k, v in
                           sorted(stats_warm.items(), key=lambda kv: -kv[1][1])},
    }
    if not args.no_plain and main_kind == zkvc.CRPC_PSQ:
        log("setup plain")
        t0 = time.perf_counter()
        pkp = zkvc.setup(a, n, b, zkvc.PLAIN, tox)
        setup_plain = time.perf_counter() - t0
        steps_p = max(3, args.steps // 3)
        log(f"timing {steps_p} plain proofs")
        tp, latp, statsp, _ = time_proofs(zkvc, lambda: zkvc.prove_device(pkp, Xd, Wd, r, s, Yd), steps_p, 2,
                                          profile=True)
        pp = zkvc.prove_device(pkp, Xd, Wd, r, s, Yd)
        okp = zkvc.verify(pkp.vk, X, Yd.cpu().numpy(), pp) == 1
        pkp.close()
        name_p, roof_p = roofline(statsp, "plain_49x320x512", mpeak)
        out["plain"] = {"workload": "same matmul, per-product circuit: 8,028,160 constraints, QAP domain 2^23",
                        "proofs_per_s": round(steps_p / tp, 3), "ms_per_proof": round(tp / steps_p * 1e3, 3),
                        "setup_s": round(setup_plain, 3), "verified": okp, "roofline": roof_p,
                        "crpc_psq_speedup": round((tp / steps_p) / (total / args.steps), 2)}
    if not args.no_msm:
        msm = {}
        for lg in (16, 20, 23, 24):
            log(f"G1 MSM 2^{lg}")
            rate, ms = msm_rate(zkvc, 1 << lg, seed)
            msm[f"2^{lg}"] = {"mpts_per_s": round(rate, 2), "ms": round(ms, 3)}
        out["msm_g1_uniform_scalars"] = msm
        msm2 = {}
        for lg in (16, 20):
            log(f"G2 MSM 2^{lg}")
            rate, ms = msm_rate(zkvc, 1 << lg, seed, group=2)
            msm2[f"2^{lg}"] = {"mpts_per_s": round(rate, 2), "ms": round(ms, 3)}
        out["msm_g2_uniform_scalars"] = msm2
        nb = SHAPE[1] * SHAPE[2]
        log(f"int8-scalar MSMs of {nb} terms (the B query)")
        r1, m1 = msm_rate(zkvc, nb, seed, group=1, int8=True)
        r2, m2 = msm_rate(zkvc, nb, seed, group=2, int8=True)
        out["msm_int8_scalars_163840"] = {"g1": {"mpts_per_s": round(r1, 2), "ms": round(m1, 3)},
                                          "g2": {"mpts_per_s": round(r2, 2), "ms": round(m2, 3)}}
        ntt = {}
        for lg in (16, 20, 24):
            log(f"NTT 2^{lg}")
            ntt[f"2^{lg}"] = ntt_rate(zkvc, lg, seed)
        out["ntt_fr_forward"] = ntt
    if not args.no_batch:
        log("batched proving: 64 mixed-shape CRPC+PSQ proofs")
        out["batched_crpc_psq_64"] = batch_section(zkvc, seed)
    if not args.no_serve:
        log("served proving: Poisson arrivals")
        out["served_crpc_psq"] = serve_section(zkvc, seed, seconds=args.serve_seconds,
                                               max_jobs=args.serve_max_jobs)
    if not args.no_table2:
        log("Table II ablation rows")
        out["table2_gpu"] = table2_section(zkvc, seed)
    if not args.no_spartan:
        log("Spartan backend (zkVC-S)")
        out["spartan_zkvc_s"] = spartan_section(zkvc, seed)
    out["paper_context"] = {"note": "the paper's CPU figures, other hardware (16-core Threadripper PRO 3955WX)",
                            "plain_prove_s_49x320x512": 180, "crpc_psq_prove_s_49x64x128_table2": 0.73}
    if not args.no_cpu_baseline:
        log("CPU oracle baseline (one whole proof on every host core)")
        out["cpu_baseline"] = cpu_baseline(X, W, tox, z, r, s)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
