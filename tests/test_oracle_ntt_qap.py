"""Pins for the oracle's transforms and QAP quotient (no GPU)."""
import random

import pytest

from oracle import ntt, qap
from oracle.bn254 import R


def _rand(n, seed):
    rng = random.Random(seed)
    return [rng.randrange(R) for _ in range(n)]


def test_roots_of_unity():
    for log_n in range(0, 29):
        n = 1 << log_n
        w = ntt.root_of_unity(n)
        assert pow(w, n, R) == 1
        if n > 1:
            assert pow(w, n // 2, R) == R - 1
    # the coset shift lies outside every domain used
    for log_n in range(0, 29):
        assert pow(ntt.COSET_SHIFT, 1 << log_n, R) != 1


@pytest.mark.parametrize("log_n", range(0, 11))
def test_fft_equals_dft(log_n):
    n = 1 << log_n
    x = _rand(n, log_n)
    w = ntt.root_of_unity(n)
    X = ntt.fft(x, w)
    assert X == ntt.dft(x, w)
    assert ntt.ifft(X, w) == x


@pytest.mark.slow
def test_fft_equals_dft_4096():
    n = 1 << 12
    x = _rand(n, 99)
    w = ntt.root_of_unity(n)
    assert ntt.fft(x, w) == ntt.dft(x, w)


def test_transform_closed_forms():
    n = 64
    w = ntt.root_of_unity(n)
    # delta at 0 -> all ones; all ones -> N delta
    delta = [1] + [0] * (n - 1)
    assert ntt.transform(delta) == [1] * n
    assert ntt.transform([1] * n) == [n] + [0] * (n - 1)
    # delta at j -> X_k = w^(jk)
    j = 5
    dj = [0] * n
    dj[j] = 1
    assert ntt.transform(dj) == [pow(w, j * k, R) for k in range(n)]
    # geometric sequence c^j -> (c^N - 1)/(c w^k - 1)
    c = 123456789
    geo = [pow(c, k, R) for k in range(n)]
    want = [(pow(c, n, R) - 1) * pow((c * pow(w, k, R) - 1) % R, -1, R) % R for k in range(n)]
    assert ntt.transform(geo) == want
    # coset forward of delta at j is g^j w^(jk)
    assert ntt.transform(dj, coset=True) == [pow(ntt.COSET_SHIFT, j, R) * pow(w, j * k, R) % R
                                             for k in range(n)]


def test_coset_round_trip_and_evaluation():
    n = 32
    x = _rand(n, 4)
    X = ntt.transform(x, coset=True)
    assert ntt.transform(X, inverse=True, coset=True) == x
    # coset forward = evaluation of the polynomial with coefficients x at g w^k
    w = ntt.root_of_unity(n)
    for k in (0, 1, 7, 31):
        pt = ntt.COSET_SHIFT * pow(w, k, R) % R
        assert X[k] == qap.poly_eval(x, pt)


def test_freivalds_check_accepts_and_rejects():
    n = 256
    x = _rand(n, 8)
    X = ntt.transform(x)
    rho = 987654321987654321
    assert ntt.freivalds_check(x, X, rho)
    bad = list(X)
    bad[17] = (bad[17] + 1) % R
    assert not ntt.freivalds_check(x, bad, rho)


def test_freivalds_parallel_agrees_with_plain_check():
    """The chunked, batch-inverted evaluation decides like the plain one: it
    accepts the DFT (computed by the O(N^2) definition) and rejects a single
    changed output, a swapped pair and a transform on the wrong root."""
    n = 64
    x = _rand(n, 21)
    X = ntt.dft(x, ntt.root_of_unity(n))
    rho = 1234567890123456789
    for workers in (1, 3):
        assert ntt.freivalds_check_parallel(x, X, rho, workers)
        bad = list(X)
        bad[n - 1] = (bad[n - 1] + 5) % R
        assert not ntt.freivalds_check_parallel(x, bad, rho, workers)
        swapped = list(X)
        swapped[3], swapped[4] = swapped[4], swapped[3]
        assert not ntt.freivalds_check_parallel(x, swapped, rho, workers)
        other = ntt.dft(x, pow(ntt.root_of_unity(n), 3, R))
        assert not ntt.freivalds_check_parallel(x, other, rho, workers)
    assert ntt.freivalds_check(x, X, rho)


def test_lagrange_closed_form_matches_product_form():
    for n in (1, 2, 4, 16, 64):
        tau = 31415926535 + n
        L = qap.lagrange_basis_at(n, tau)
        assert L == qap.lagrange_basis_at_product_form(n, tau)
        assert sum(L) % R == 1


def test_quotient_routes_agree_and_divide():
    n = 64
    rng = random.Random(2)
    # a satisfied system: pick aev, bev freely, cev = aev*bev pointwise
    aev = [rng.randrange(R) for _ in range(n)]
    bev = [rng.randrange(R) for _ in range(n)]
    cev = [a * b % R for a, b in zip(aev, bev)]
    h1 = qap.quotient_schoolbook(aev, bev, cev)
    h2 = qap.quotient_coset(aev, bev, cev, method="dft")
    h3 = qap.quotient_coset(aev, bev, cev, method="fft")
    assert h1 == h2 == h3
    assert len(h1) == n - 1
    # h(x) t(x) = A(x) B(x) - C(x) at a random point
    w = ntt.root_of_unity(n)
    A, B, C = (ntt.idft(v, w) for v in (aev, bev, cev))
    x = 271828182845904523536
    lhs = qap.poly_eval(h1, x) * (pow(x, n, R) - 1) % R
    rhs = (qap.poly_eval(A, x) * qap.poly_eval(B, x) - qap.poly_eval(C, x)) % R
    assert lhs == rhs
    # an unsatisfied row makes the division fail on both routes
    cev[3] = (cev[3] + 1) % R
    with pytest.raises(ValueError):
        qap.quotient_schoolbook(aev, bev, cev)
    with pytest.raises(ValueError):
        qap.quotient_coset(aev, bev, cev)


def test_divide_by_vanishing_small():
    # (x^4 - 1)(x^2 + 3) = x^6 + 3x^4 - x^2 - 3
    p = [(-3) % R, 0, (-1) % R, 0, 3, 0, 1]
    q, rem = qap.divide_by_vanishing(p, 4)
    assert q == [3, 0, 1] and not any(rem)
