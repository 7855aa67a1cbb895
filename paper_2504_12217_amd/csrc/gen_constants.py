"""Writes csrc/constants.hpp: BN254 moduli and Montgomery constants for the library.

Run by the package build before compiling.  Everything is derived from the
BN curve parameter u (p and r are the BN family polynomials evaluated at u).

Two Montgomery representations are emitted:
  * device: 9 limbs of 29 bits, R = 2^261 (one 64-bit multiply-add per
    partial product, carries deferred to the column end);
  * host:   4 limbs of 64 bits, R = 2^256 (the verifier and proof assembly).
"""
import os
import sys

U = 4965661367192848881
P = 36 * U**4 + 36 * U**3 + 24 * U**2 + 6 * U + 1
R = 36 * U**4 + 36 * U**3 + 18 * U**2 + 6 * U + 1

DEV_LIMBS, DEV_BITS = 9, 29
DEV_R = 1 << (DEV_LIMBS * DEV_BITS)
HOST_R = 1 << 256


def limbs(v, n, bits):
    return [(v >> (bits * k)) & ((1 << bits) - 1) for k in range(n)]


def arr(name, vals, ctype, fmt):
    body = ", ".join(fmt.format(v) for v in vals)
    return f"static constexpr {ctype} {name}[{len(vals)}] = {{{body}}};"


def field_block(tag, m):
    dev_pinv = (-pow(m, -1, 1 << DEV_BITS)) % (1 << DEV_BITS)
    host_pinv = (-pow(m, -1, 1 << 64)) % (1 << 64)
    lines = [
        f"struct {tag}Params {{",
        "  " + arr("P", limbs(m, DEV_LIMBS, DEV_BITS), "uint32_t", "0x{:08x}u"),
        "  " + arr("P2", limbs(2 * m, DEV_LIMBS, DEV_BITS), "uint32_t", "0x{:08x}u"),
        "  " + arr("P4", limbs(4 * m, DEV_LIMBS, DEV_BITS), "uint32_t", "0x{:08x}u"),
        "  " + arr("P6", limbs(6 * m, DEV_LIMBS, DEV_BITS), "uint32_t", "0x{:08x}u"),
        f"  static constexpr uint32_t PINV = 0x{dev_pinv:08x}u;  // -m^-1 mod 2^29",
        "  " + arr("ONE", limbs(DEV_R % m, DEV_LIMBS, DEV_BITS), "uint32_t", "0x{:08x}u") + "  // 2^261 mod m",
        "  " + arr("R2", limbs(DEV_R * DEV_R % m, DEV_LIMBS, DEV_BITS), "uint32_t", "0x{:08x}u") + "  // 2^522 mod m",
        "  " + arr("P32", limbs(m, 8, 32), "uint32_t", "0x{:08x}u"),
        "  " + arr("HALF32", limbs((m - 1) // 2, 8, 32), "uint32_t", "0x{:08x}u") + "  // (m-1)/2",
        "  " + arr("P64", limbs(m, 4, 64), "uint64_t", "0x{:016x}ull"),
        f"  static constexpr uint64_t PINV64 = 0x{host_pinv:016x}ull;  // -m^-1 mod 2^64",
        "  " + arr("ONE64", limbs(HOST_R % m, 4, 64), "uint64_t", "0x{:016x}ull") + "  // 2^256 mod m",
        "  " + arr("R2_64", limbs(HOST_R * HOST_R % m, 4, 64), "uint64_t", "0x{:016x}ull") + "  // 2^512 mod m",
        "  " + arr("DEVR_64", limbs(DEV_R % m, 4, 64), "uint64_t", "0x{:016x}ull") + "  // 2^261 mod m (canonical)",
        "};",
    ]
    return "\n".join(lines)


# Standard BN254 G2 generator on the twist y^2 = x^3 + 3/(9+i), x = x0 + x1 i.
G2_X0 = 10857046999023057135944570762232829481370756359578518086990519993285655852781
G2_X1 = 11559732032986387107991004021392285783925812861821192530917403151452391805634
G2_Y0 = 8495653923123431417604973247489272438418190587263600148770280649306958101930
G2_Y1 = 4082367875863433681332203403145435568316851327593401208105741076214120093531


def cube_root_of_unity(m):
    """A primitive cube root of unity mod the prime m (m = 1 mod 3)."""
    for g in range(2, 100):
        w = pow(g, (m - 1) // 3, m)
        if w != 1:
            return w
    raise ValueError("no cube root found")


def affine_add(p1, p2):
    """Sum of two points of y^2 = x^3 + 3 over Fq (None is infinity)."""
    if p1 is None:
        return p2
    if p2 is None:
        return p1
    (x1, y1), (x2, y2) = p1, p2
    if x1 == x2:
        if (y1 + y2) % P == 0:
            return None
        slope = 3 * x1 * x1 * pow(2 * y1, -1, P) % P
    else:
        slope = (y2 - y1) * pow(x2 - x1, -1, P) % P
    x3 = (slope * slope - x1 - x2) % P
    return (x3, (slope * (x1 - x3) - y1) % P)


def affine_mul(k, pt):
    acc = None
    for bit in bin(k)[2:]:
        acc = affine_add(acc, acc)
        if bit == "1":
            acc = affine_add(acc, pt)
    return acc


def glv_block():
    """G1 endomorphism phi(x, y) = (beta x, y) = lambda (x, y) and a short basis
    of the lattice {(a, b): a + b lambda = 0 mod r} (Gallant, Lambert and
    Vanstone, CRYPTO 2001), from the extended Euclidean algorithm on (r, lambda)."""
    w_p, w_r = cube_root_of_unity(P), cube_root_of_unity(R)
    gen = (1, 2)
    pairs = [(b, l) for b in (w_p, w_p * w_p % P) for l in (w_r, w_r * w_r % R)
             if affine_mul(l, gen) == (b * gen[0] % P, gen[1])]
    assert len(pairs) == 2  # (beta, lambda) and (beta^2, lambda^2)
    beta, lam = min(pairs)
    seq = [(R, 0), (lam, 1)]
    while seq[-1][0]:
        (r0, t0), (r1, t1) = seq[-2], seq[-1]
        q = r0 // r1
        seq.append((r0 - q * r1, t0 - q * t1))
    root = 1
    while root * root <= R:
        root *= 2
    lo, hi = root // 2, root  # integer square root by bisection
    while hi - lo > 1:
        mid = (lo + hi) // 2
        lo, hi = (mid, hi) if mid * mid <= R else (lo, mid)
    m = max(i for i, (ri, _) in enumerate(seq) if ri >= lo)
    v1 = (seq[m + 1][0], -seq[m + 1][1])
    v2 = min((seq[m][0], -seq[m][1]), (seq[m + 2][0], -seq[m + 2][1]), key=lambda v: v[0] ** 2 + v[1] ** 2)
    (a1, b1), (a2, b2) = v1, v2
    for a, b in (v1, v2):
        assert (a + b * lam) % R == 0
    # the signs the host decomposition is written for
    assert a1 > 0 and b1 < 0 and a2 > 0 and b2 > 0 and a1 * b2 - a2 * b1 == R
    g1, g2 = (b2 << 256) // R, ((-b1) << 256) // R
    return "\n".join([
        "// G1 endomorphism (x, y) -> (beta x, y), equal to multiplication by lambda,",
        "// and the short lattice basis v1 = (A1, -B1ABS), v2 = (A2, B2) of",
        "// {(a, b): a + b lambda = 0 mod r}; G1C = floor(B2 2^256 / r),",
        "// G2C = floor(B1ABS 2^256 / r).",
        "struct G1Glv {",
        f"  // lambda = {lam}",
        "  " + arr("BETA", limbs(beta, 4, 64), "uint64_t", "0x{:016x}ull") + "  // canonical",
        "  " + arr("A1", limbs(a1, 4, 64), "uint64_t", "0x{:016x}ull"),
        "  " + arr("B1ABS", limbs(-b1, 4, 64), "uint64_t", "0x{:016x}ull"),
        "  " + arr("A2", limbs(a2, 4, 64), "uint64_t", "0x{:016x}ull"),
        "  " + arr("B2", limbs(b2, 4, 64), "uint64_t", "0x{:016x}ull"),
        "  " + arr("G1C", limbs(g1, 4, 64), "uint64_t", "0x{:016x}ull"),
        "  " + arr("G2C", limbs(g2, 4, 64), "uint64_t", "0x{:016x}ull"),
        "};",
    ])


def main(out_path):
    assert P + 1 - (6 * U * U + 1) == R
    text = "\n".join([
        "// Generated by gen_constants.py from the BN254 parameter u; do not edit.",
        "#pragma once",
        "#include <cstdint>",
        "namespace zkvc {",
        f"// u = {U}",
        f"// p = {P}",
        f"// r = {R}",
        field_block("Fq", P),
        field_block("Fr", R),
        "struct G2Gen {",
        "  " + arr("X0", limbs(G2_X0, 4, 64), "uint64_t", "0x{:016x}ull"),
        "  " + arr("X1", limbs(G2_X1, 4, 64), "uint64_t", "0x{:016x}ull"),
        "  " + arr("Y0", limbs(G2_Y0, 4, 64), "uint64_t", "0x{:016x}ull"),
        "  " + arr("Y1", limbs(G2_Y1, 4, 64), "uint64_t", "0x{:016x}ull"),
        "};",
        glv_block(),
        "}  // namespace zkvc",
        "",
    ])
    old = open(out_path).read() if os.path.exists(out_path) else None
    if old != text:
        with open(out_path, "w") as f:
            f.write(text)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else os.path.join(os.path.dirname(__file__), "constants.hpp"))
