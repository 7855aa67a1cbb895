"""Number-theoretic transforms over Fr for the CPU oracle.

TEST INFRASTRUCTURE ONLY (see oracle/bn254.py).

The QAP is obtained from the R1CS by interpolation over a domain (Section II,
ZKP systems); the quotient h(x) is found by moving between evaluations on the
domain, coefficients, and evaluations on a coset.  This module provides:

  * dft / idft: the O(N^2) definitions  X_k = sum_j x_j w^(jk)  and
    x_j = N^-1 sum_k X_k w^(-jk);
  * fft / ifft: a textbook recursive radix-2 Cooley-Tukey FFT, used where the
    O(N^2) sums are too slow; the tests prove fft == dft for every power of
    two up to 2^12 before anything relies on it;
  * the coset variants (input scaled by g^j before the forward transform,
    output scaled by g^-j after the inverse).

Domain convention: omega_N = 5^((r-1)/N) (5 generates Fr^*, r - 1 has
2-adicity 28), coset shift g = 5.
"""
from .bn254 import R

TWO_ADICITY = 28
GENERATOR = 5
COSET_SHIFT = 5


def root_of_unity(n):
    """Primitive n-th root of unity in Fr for n a power of two <= 2^28."""
    if n <= 0 or n & (n - 1) or n > (1 << TWO_ADICITY):
        raise ValueError("n must be a power of two <= 2^28")
    return pow(GENERATOR, (R - 1) // n, R)


def dft(x, omega):
    n = len(x)
    out = []
    for k in range(n):
        wk = pow(omega, k, R)
        acc = 0
        wkj = 1
        for j in range(n):
            acc += x[j] * wkj
            wkj = wkj * wk % R
        out.append(acc % R)
    return out


def idft(X, omega):
    n = len(X)
    inv_n = pow(n, -1, R)
    return [v * inv_n % R for v in dft(X, pow(omega, -1, R))]


def fft(x, omega):
    """Recursive radix-2 decimation-in-time FFT: X_k = sum_j x_j omega^(jk)."""
    n = len(x)
    if n == 1:
        return [x[0] % R]
    even = fft(x[0::2], omega * omega % R)
    odd = fft(x[1::2], omega * omega % R)
    out = [0] * n
    w = 1
    half = n // 2
    for k in range(half):
        t = w * odd[k] % R
        out[k] = (even[k] + t) % R
        out[k + half] = (even[k] - t) % R
        w = w * omega % R
    return out


def ifft(X, omega):
    n = len(X)
    inv_n = pow(n, -1, R)
    return [v * inv_n % R for v in fft(X, pow(omega, -1, R))]


def transform(x, inverse=False, coset=False, method="fft"):
    """Natural-order NTT of len(x) = N elements, as the library's flags define it.

    forward:          X_k = sum_j (g^j if coset else 1) x_j omega^(jk)
    inverse:          x_j = (g^-j if coset else 1) N^-1 sum_k X_k omega^(-jk)
    """
    n = len(x)
    omega = root_of_unity(n)
    f, finv = (fft, ifft) if method == "fft" else (dft, idft)
    if not inverse:
        if coset:
            x = [v * pow(COSET_SHIFT, j, R) % R for j, v in enumerate(x)]
        return f(x, omega)
    out = finv(x, omega)
    if coset:
        ginv = pow(COSET_SHIFT, -1, R)
        out = [v * pow(ginv, j, R) % R for j, v in enumerate(out)]
    return out


def freivalds_check(x, X, rho):
    """Probabilistic check that X = NTT(x) on a domain of size N.

    For any rho outside the domain,
        sum_k X_k rho^k = sum_j x_j sum_k (rho omega^j)^k
                        = sum_j x_j (rho^N - 1) / (rho omega^j - 1).
    A wrong X passes for at most N of the r possible rho.
    """
    n = len(x)
    omega = root_of_unity(n)
    lhs = 0
    rk = 1
    for v in X:
        lhs = (lhs + v * rk) % R
        rk = rk * rho % R
    rn1 = (pow(rho, n, R) - 1) % R
    rhs = 0
    wj = 1
    for v in x:
        rhs = (rhs + v * pow((rho * wj - 1) % R, -1, R)) % R
        wj = wj * omega % R
    return lhs == rhs * rn1 % R


_FV = {}


def _freivalds_part(job):
    """Partial sums of the two sides of the Freivalds identity over indices [k0, k1)."""
    k0, k1, rho, omega = job
    x, X = _FV["x"], _FV["X"]
    # left: sum_k X_k rho^k
    lhs = 0
    rk = pow(rho, k0, R)
    for k in range(k0, k1):
        lhs = (lhs + X[k] * rk) % R
        rk = rk * rho % R
    # right: sum_j x_j / (rho omega^j - 1), the denominators inverted together
    # (prefix products, one inversion, then back substitution)
    dens = []
    wj = pow(omega, k0, R)
    for _ in range(k0, k1):
        dens.append((rho * wj - 1) % R)
        wj = wj * omega % R
    pre = [1] * len(dens)
    acc = 1
    for i, d in enumerate(dens):
        pre[i] = acc
        acc = acc * d % R
    inv = pow(acc, -1, R)
    rhs = 0
    for i in range(len(dens) - 1, -1, -1):
        rhs = (rhs + x[k0 + i] * (inv * pre[i] % R)) % R
        inv = inv * dens[i] % R
    return lhs, rhs


def freivalds_check_parallel(x, X, rho, workers=1):
    """freivalds_check with the sums split into index ranges (over `workers`
    processes if > 1) and the denominators of each range inverted together:
    the same identity, evaluated at O(N) field cost with N / chunk inversions.
    rho must lie outside the domain (rho omega^j != 1 for every j)."""
    n = len(x)
    omega = root_of_unity(n)
    step = max(1, -(-n // max(1, 4 * workers)))
    jobs = [(k0, min(n, k0 + step), rho, omega) for k0 in range(0, n, step)]
    _FV["x"], _FV["X"] = x, X
    try:
        if workers <= 1:
            parts = [_freivalds_part(j) for j in jobs]
        else:
            import multiprocessing as mp
            with mp.get_context("fork").Pool(workers) as pool:
                parts = pool.map(_freivalds_part, jobs)
    finally:
        _FV.clear()
    lhs = sum(p[0] for p in parts) % R
    rhs = sum(p[1] for p in parts) % R
    return lhs == rhs * ((pow(rho, n, R) - 1) % R) % R
