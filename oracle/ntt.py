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
