"""The host's G1 scalar multiplication by the endomorphism (x, y) -> (beta x, y)
(Gallant-Lambert-Vanstone), which the prover uses for s A + r B1 when it
assembles C (Groth16's prover, §II): checked against the oracle's double-and-add
on random and edge scalars, with the split k = k1 + k2 lambda (mod r) and
|k1|, |k2| < 2^128 checked on every case.  No GPU: the host code is built alone."""
import os
import random
import shutil
import subprocess

import pytest

from oracle import bn254 as bn

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2504_12217_amd", "csrc")


def _lambda():
    # the cube root of unity in Fr by which phi acts on G1, read from the pair
    # (beta, lambda) the generator satisfies: phi(G) = lambda G
    for g in range(2, 50):
        w = pow(g, (bn.R - 1) // 3, bn.R)
        if w != 1:
            break
    for lam in (w, w * w % bn.R):
        x, y = bn.g1_mul(bn.G1_GEN, lam)
        if y == bn.G1_GEN[1] and pow(x, 3, bn.P) == 1 and x != 1:
            return lam
    raise AssertionError("no lambda")


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    cxx = shutil.which("g++") or shutil.which("clang++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("glv") / "host_glv_check")
    subprocess.run([cxx, "-O2", "-std=c++17", "-I", CSRC, os.path.join(HERE, "host_glv_check.cpp"), "-o", exe],
                   check=True)
    return exe


def _hex(v):
    return format(v, "x")


def test_glv_matches_double_and_add(harness):
    rng = random.Random(20250417)
    lam = _lambda()
    P = bn.g1_mul(bn.G1_GEN, 7)
    Q = bn.g1_mul(bn.G1_GEN, 1234567)
    ks = [0, 1, 2, bn.R - 1, bn.R - 2, lam, bn.R - lam, (bn.R - 1) // 2, 1 << 127, (1 << 128) - 1]
    ks += [rng.randrange(bn.R) for _ in range(60)]
    bs = [rng.randrange(bn.R) for _ in ks]
    bs[1] = 0
    lines = "".join(f"{_hex(P[0])} {_hex(P[1])} {_hex(Q[0])} {_hex(Q[1])} {_hex(k)} {_hex(b)}\n"
                    for k, b in zip(ks, bs))
    out = subprocess.run([harness], input=lines, capture_output=True, text=True, check=True).stdout.split("\n")
    for k, b, line in zip(ks, bs, out):
        f = line.split()
        kp = None if f[0] == "inf" else (int(f[0], 16), int(f[1], 16))
        kpbq = None if f[2] == "inf" else (int(f[2], 16), int(f[3], 16))
        assert kp == bn.g1_mul(P, k), k
        assert kpbq == bn.g1_add(bn.g1_mul(P, k), bn.g1_mul(Q, b)), (k, b)
        k1 = (-1 if f[4] == "1" else 1) * int(f[5], 16)
        k2 = (-1 if f[6] == "1" else 1) * int(f[7], 16)
        assert (k1 + k2 * lam - k) % bn.R == 0
        assert abs(k1) < 1 << 128 and abs(k2) < 1 << 128
