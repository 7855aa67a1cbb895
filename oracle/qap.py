"""R1CS -> QAP and the quotient polynomial h(x), for the CPU oracle.

TEST INFRASTRUCTURE ONLY (see oracle/bn254.py).

The QAP comes from the R1CS by interpolation over the domain
H = {omega^c : c < N} (Section II, ZKP systems).  Row c of the constraint
system sits at omega^c.  With L_c the Lagrange basis of H,
    u_i(x) = sum_c A[c][i] L_c(x),  v_i likewise from B,  w_i from C,
and for an assignment a
    A(x) = sum_i a_i u_i(x) = sum_c <A_c, a> L_c(x)   (B, C likewise).
The assignment satisfies the R1CS iff t(x) = x^N - 1 divides A B - C, and the
quotient h = (A B - C) / t has degree at most N - 2.

Two independent routes to h are provided:
  * quotient_schoolbook: interpolate by the O(N^2) inverse DFT, multiply the
    polynomials coefficient by coefficient, and divide by x^N - 1 by long
    division (this is the definition; used for small N);
  * quotient_coset: the FFT route (inverse transform to coefficients, forward
    transform on the coset g H where t does not vanish, pointwise
    (A B - C) / t(g omega^k) with t(g omega^k) = g^N - 1, inverse coset
    transform), which is what a fast prover does.
"""
from .bn254 import R
from . import ntt
from . import r1cs


def lagrange_basis_at(n, tau):
    """[L_c(tau) for c < n] with L_c(x) = omega^c (x^n - 1) / (n (x - omega^c)).

    The closed form follows from prod_{k != c} (x - omega^k) = (x^n - 1)/(x - omega^c)
    and its value n omega^-c at x = omega^c.  tau must lie outside the domain.
    """
    omega = ntt.root_of_unity(n)
    tn1 = (pow(tau, n, R) - 1) % R
    if tn1 == 0:
        raise ValueError("tau lies in the evaluation domain")
    inv_n = pow(n, -1, R)
    out = []
    wc = 1
    for _ in range(n):
        out.append(wc * tn1 % R * inv_n % R * pow((tau - wc) % R, -1, R) % R)
        wc = wc * omega % R
    return out


def lagrange_basis_range(n, tau, c0, c1):
    """[L_c(tau) for c0 <= c < c1] by the same closed form as lagrange_basis_at."""
    omega = ntt.root_of_unity(n)
    tn1 = (pow(tau, n, R) - 1) % R
    if tn1 == 0:
        raise ValueError("tau lies in the evaluation domain")
    k = tn1 * pow(n, -1, R) % R
    out = []
    wc = pow(omega, c0, R)
    for _ in range(c0, c1):
        out.append(wc * k % R * pow((tau - wc) % R, -1, R) % R)
        wc = wc * omega % R
    return out


def lagrange_basis_at_product_form(n, tau):
    """L_c(tau) = prod_{k != c} (tau - omega^k) / (omega^c - omega^k); O(n^2), for pins."""
    omega = ntt.root_of_unity(n)
    pts = [pow(omega, k, R) for k in range(n)]
    out = []
    for c in range(n):
        num, den = 1, 1
        for k in range(n):
            if k != c:
                num = num * (tau - pts[k]) % R
                den = den * (pts[c] - pts[k]) % R
        out.append(num * pow(den, -1, R) % R)
    return out


def var_polys_at(s, kind, tau, z=None):
    """u_i(tau), v_i(tau), w_i(tau) for every variable i."""
    n_dom = r1cs.domain_size(s, kind)
    L = lagrange_basis_at(n_dom, tau)
    nv = r1cs.num_vars(s, kind)
    u, v, w = [0] * nv, [0] * nv, [0] * nv
    for c, (A, B, C) in enumerate(r1cs.rows(s, kind, z)):
        for i, coef in A.items():
            u[i] = (u[i] + coef * L[c]) % R
        for i, coef in B.items():
            v[i] = (v[i] + coef * L[c]) % R
        for i, coef in C.items():
            w[i] = (w[i] + coef * L[c]) % R
    return u, v, w


_SHARED = {}


def _var_poly_part(job):
    s, kind, zp, tau, n_dom, c0, c1 = job
    want = _SHARED["vars"]
    L = lagrange_basis_range(n_dom, tau, c0, c1)
    acc = {}
    for c in range(c0, c1):
        for q, row in enumerate(r1cs.row(s, kind, c, zp)):
            for i, coef in row.items():
                if i in want:
                    key = (q, i)
                    acc[key] = (acc.get(key, 0) + coef * L[c - c0]) % R
    return acc


def var_polys_sampled(s, kind, tau, variables, z=None, workers=1):
    """{i: (u_i(tau), v_i(tau), w_i(tau))} for the listed variables only.

    The same row sums as var_polys_at, restricted to a sample of variables and
    optionally split over processes by row range.
    """
    n_dom = r1cs.domain_size(s, kind)
    zp = r1cs.z_powers(s, z) if kind in r1cs.CRPC_KINDS else None
    nrows = r1cs.num_constraints(s, kind) + r1cs.num_public(s) + 1
    _SHARED["vars"] = set(variables)
    if workers <= 1:
        parts = [_var_poly_part((s, kind, zp, tau, n_dom, 0, nrows))]
    else:
        import multiprocessing as mp
        step = -(-nrows // (workers * 4))
        jobs = [(s, kind, zp, tau, n_dom, c, min(c + step, nrows)) for c in range(0, nrows, step)]
        with mp.get_context("fork").Pool(workers) as pool:
            parts = pool.map(_var_poly_part, jobs)
    _SHARED.clear()
    out = {i: [0, 0, 0] for i in variables}
    for part in parts:
        for (q, i), v in part.items():
            out[i][q] = (out[i][q] + v) % R
    return {i: tuple(v) for i, v in out.items()}


def poly_mul(a, b):
    out = [0] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        if x:
            for j, y in enumerate(b):
                out[i + j] += x * y
    return [c % R for c in out]


def poly_eval(coeffs, x):
    acc = 0
    for c in reversed(coeffs):
        acc = (acc * x + c) % R
    return acc


def divide_by_vanishing(p, n):
    """Quotient and remainder of p(x) / (x^n - 1)."""
    rem = list(p) + [0] * max(0, n - len(p))
    q = [0] * max(len(p) - n, 0)
    for d in range(len(rem) - 1, n - 1, -1):
        c = rem[d] % R
        if c:
            q[d - n] = c
            rem[d] = 0
            rem[d - n] = (rem[d - n] + c) % R
    return q, [c % R for c in rem[:n]]


def quotient_schoolbook(aev, bev, cev):
    """h by definition: interpolate, multiply, long-divide by x^N - 1 (small N only)."""
    n = len(aev)
    omega = ntt.root_of_unity(n)
    A = ntt.idft(aev, omega)
    B = ntt.idft(bev, omega)
    C = ntt.idft(cev, omega)
    AB = poly_mul(A, B)
    num = [(AB[k] - (C[k] if k < n else 0)) % R for k in range(len(AB))]
    q, rem = divide_by_vanishing(num, n)
    if any(rem):
        raise ValueError("A*B - C is not divisible by x^N - 1: the R1CS is not satisfied")
    q = q + [0] * (n - 1 - len(q))
    return q[: n - 1]


def quotient_coset(aev, bev, cev, method="fft"):
    """h by the coset route; returns h_0..h_{N-2} and asserts h_{N-1} = 0."""
    n = len(aev)
    A = ntt.transform(aev, inverse=True, method=method)
    B = ntt.transform(bev, inverse=True, method=method)
    C = ntt.transform(cev, inverse=True, method=method)
    Ae = ntt.transform(A, coset=True, method=method)
    Be = ntt.transform(B, coset=True, method=method)
    Ce = ntt.transform(C, coset=True, method=method)
    zinv = pow((pow(ntt.COSET_SHIFT, n, R) - 1) % R, -1, R)
    q = [(x * y - c) * zinv % R for x, y, c in zip(Ae, Be, Ce)]
    h = ntt.transform(q, inverse=True, coset=True, method=method)
    if h[n - 1] != 0:
        raise ValueError("h has degree N-1: the R1CS is not satisfied")
    return h[: n - 1]
