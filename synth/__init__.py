"""Seeded synthetic inputs for the matmul prover.

This module is the only code that the CPU oracle and the GPU library's tests
and benchmark both use.  It holds none of the prover's arithmetic: it draws
integers and reports them as numpy arrays.

Every draw comes from numpy's PCG64 seeded with SeedSequence([seed, stream]),
one stream per purpose, so results do not depend on call order:

    1 X matrix   2 W matrix   3 toxic waste   4 CRPC point z   5 prover (r, s)
    6 MSM scalars   7 MSM base logarithms   8 NTT inputs   9 arrivals   10 shapes

Quantized activations and weights are stood in for by int8 entries uniform in
[-128, 127] (the paper quantizes model parameters to integers, Section IV,
without giving the bit width).  Field elements are uniform in [0, r) for the
BN254 scalar field order r, drawn by rejection from 254-bit words and
returned as 8 little-endian 32-bit limbs.
"""
import numpy as np

STREAM_X, STREAM_W, STREAM_TOXIC, STREAM_Z, STREAM_RS = 1, 2, 3, 4, 5
STREAM_MSM_SCALARS, STREAM_MSM_BASES, STREAM_NTT, STREAM_ARRIVALS, STREAM_SHAPES = 6, 7, 8, 9, 10

# BN254 scalar field order: only used as the upper bound of uniform draws.
FR_ORDER = 21888242871839275222246405745257275088548364400416034343698204186575808495617
_FR_WORDS = np.array([(FR_ORDER >> (64 * k)) & 0xFFFFFFFFFFFFFFFF for k in range(4)], dtype=np.uint64)


def rng(seed, stream):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(stream)])))


def int8_matrix(seed, stream, rows, cols):
    """rows x cols int8 matrix, entries uniform in [-128, 127]."""
    g = rng(seed, stream)
    raw = g.bit_generator.random_raw(rows * cols)
    return ((raw & np.uint64(0xFF)).astype(np.int16) - 128).astype(np.int8).reshape(rows, cols)


def matmul_inputs(seed, a, n, b):
    """(X [a, n], W [n, b]) int8 for one proof job."""
    return int8_matrix(seed, STREAM_X, a, n), int8_matrix(seed, STREAM_W, n, b)


def _below_order(w):
    """Row-wise test w < FR_ORDER for an [m, 4] uint64 array (little-endian words)."""
    lt = np.zeros(w.shape[0], dtype=bool)
    eq = np.ones(w.shape[0], dtype=bool)
    for k in (3, 2, 1, 0):
        lt |= eq & (w[:, k] < _FR_WORDS[k])
        eq &= w[:, k] == _FR_WORDS[k]
    return lt


def fr_limbs(seed, stream, count):
    """[count, 8] uint32 little-endian limbs of elements uniform in [0, r)."""
    g = rng(seed, stream)
    out = np.empty((count, 4), dtype=np.uint64)
    filled = 0
    while filled < count:
        need = count - filled
        m = need + need // 3 + 16
        w = g.bit_generator.random_raw(4 * m).reshape(m, 4)
        w[:, 3] &= np.uint64((1 << 62) - 1)  # 254-bit words
        ok = w[_below_order(w)]
        take = min(need, ok.shape[0])
        out[filled:filled + take] = ok[:take]
        filled += take
    return out.view(np.uint32).reshape(count, 8)


def limbs_to_ints(limbs):
    """Python ints from [m, 8] uint32 little-endian limbs."""
    b = np.ascontiguousarray(limbs, dtype=np.uint32).tobytes()
    return [int.from_bytes(b[32 * i:32 * i + 32], "little") for i in range(len(b) // 32)]


def ints_to_limbs(values):
    """[m, 8] uint32 limbs from Python ints in [0, 2^256)."""
    b = b"".join(int(v).to_bytes(32, "little") for v in values)
    return np.frombuffer(b, dtype=np.uint32).reshape(-1, 8).copy()


def nonzero_fr(seed, stream, count):
    """count nonzero field elements (as Python ints), redrawing zeros."""
    vals = [v for v in limbs_to_ints(fr_limbs(seed, stream, count + 4)) if v != 0]
    return vals[:count]


def toxic_waste(seed):
    """(tau, alpha, beta, gamma, delta), each a nonzero element of Fr."""
    return tuple(nonzero_fr(seed, STREAM_TOXIC, 5))


def crpc_point(seed):
    """The public CRPC evaluation point z (nonzero)."""
    return nonzero_fr(seed, STREAM_Z, 1)[0]


def prover_randomness(seed, job=0):
    """(r, s) blinding scalars for proof job `job`."""
    vals = limbs_to_ints(fr_limbs(seed * 1000003 + job, STREAM_RS, 2))
    return vals[0], vals[1]


def exponential_gaps(seed, rate, count):
    """Inter-arrival gaps (seconds) of a Poisson process of the given rate."""
    g = rng(seed, STREAM_ARRIVALS)
    u = (g.bit_generator.random_raw(count) >> np.uint64(11)).astype(np.float64) * 2.0**-53
    return -np.log1p(-u) / rate


# ---------------------------------------------------------------- workload mixes
# The paper's matmul shapes are [#tokens, dim1] x [dim1, dim2] with 49 tokens
# (Section IV); the headline is [49, 320] x [320, 512] (Section I).
TOKENS = 49
PAPER_SHAPE = (49, 320, 512)
BATCH_N = (64, 128, 320)
BATCH_B = (64, 256, 512)


def batch_jobs(seed, count):
    """A batch of mixed-shape proof jobs: (shape, X, W, r, s) per job.

    (n, b) of job j is class (word_j mod 9) of {64,128,320} x {64,256,512}
    (stream 10), a = 49; X, W of job j come from seed 1000 seed + j + 1 and
    (r, s) from prover_randomness(seed, job=j)."""
    raw = rng(seed, STREAM_SHAPES).bit_generator.random_raw(count)
    shapes = [(TOKENS, BATCH_N[int(w % 9) // 3], BATCH_B[int(w % 9) % 3]) for w in raw]
    jobs = []
    for j, (a, n, b) in enumerate(shapes):
        X, W = matmul_inputs(1000 * seed + j + 1, a, n, b)
        r, s = prover_randomness(seed, job=j)
        jobs.append(((a, n, b), X, W, r, s))
    return jobs


def served_classes():
    """The ten shape classes of served proving: the nine batch classes, then the paper shape."""
    return [(TOKENS, n, b) for n in BATCH_N for b in BATCH_B] + [PAPER_SHAPE]


def served_jobs(seed, rate, count):
    """Poisson arrivals of proof jobs at `rate` per second over the served classes
    (equal weights): (gaps in seconds, [(shape, X, W, r, s)])."""
    classes = served_classes()
    gaps = exponential_gaps(seed + rate, rate, count)
    pick = rng(seed + rate, STREAM_SHAPES).bit_generator.random_raw(count)
    jobs = []
    for j in range(count):
        sh = classes[int(pick[j] % len(classes))]
        X, W = matmul_inputs(10000 * seed + 1000 * rate + j + 1, *sh)
        r, s = prover_randomness(seed + rate, job=j)
        jobs.append((sh, X, W, r, s))
    return gaps, jobs
