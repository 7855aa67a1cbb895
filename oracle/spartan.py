"""Spartan for the matmul constraint systems (zkVC-S), for the CPU oracle.

TEST INFRASTRUCTURE ONLY (see oracle/bn254.py).

The paper's second backend is Spartan, a transparent SNARK built from an
interactive proof over multilinear polynomials and a polynomial commitment
(Section II; Section IV names it as the zkVC-S backend, Table II gives its
prove and verify times next to Groth16's).  The paper fixes neither the
commitment scheme nor the curve, so this oracle takes these readings:

  * field: the BN254 scalar field Fr; commitments: BN254 G1;
  * the argument is Spartan's NIZK with a linear-time verifier: two sum-check
    protocols reduce R1CS satisfiability to one evaluation of the witness's
    multilinear extension, and the verifier evaluates the constraint
    matrices' extensions itself (no commitment to the matrices);
  * the witness is committed row by row with Pedersen vector commitments
    (the square-root layout of Hyrax) under generators the caller supplies,
    without blinding: the argument is succinct but not zero-knowledge;
  * Fiat-Shamir with SHA-256 over a byte transcript defined below.

Definitions (every index's bit k is variable k, least significant first):

  eq(r, b)      = prod_k (r_k b_k + (1 - r_k)(1 - b_k))
  f~(r)         = sum_i f[i] eq(r, bits(i))        (multilinear extension)
  rows          : the m multiplication constraints of the R1CS (the Groth16
                  input-consistency rows are not part of it), padded to 2^sx
  z             : length 2^sy, z[j] = a[l + 1 + j] for the witness variables
                  (the W entries, then the auxiliary ones), and
                  z[2^(sy-1) + t] = a[t] for t = 0..l (constant, x, y)
  matrix M_rx   : M(y) = sum_x eq(r_x, x) (rA A[x][y] + rB B[x][y] + rC C[x][y])

Prover:
  1. W matrix: the witness half of z as rows x cols (index = row cols + col);
     commitment C_i = sum_col w[i, col] G_col for every row i.
  2. transcript: shape and z, the public X and Y, the commitments;
     tau_0..tau_{sx-1}.
  3. sum-check 1 of sum_x eq(tau, x) (Az(x) Bz(x) - Cz(x)) = 0, degree 3:
     per round the values at 0, 1, 2, 3 of the round polynomial; the arrays
     fold on the least significant variable: f[i] <- f[2i] + r (f[2i+1] - f[2i]).
  4. vA, vB, vC = Az~(r_x), Bz~(r_x), Cz~(r_x); rA, rB, rC from the transcript.
  5. sum-check 2 of sum_y M(y) z(y) = rA vA + rB vB + rC vC, degree 2 (values
     at 0, 1, 2).
  6. opening of w~ at r' = r_y without its top coordinate: with r' split into
     column coordinates (the low ones) and row coordinates,
     t[col] = sum_row eq(r_row, row) w[row, col].
Verifier: the sum-check relations round by round; eq(tau, r_x)(vA vB - vC)
equals the last claim of sum-check 1; with v_w = <t, eq(r_col, .)> and the
public part p~(r') computed from the public inputs,
M~(r_y) ((1 - r_top) v_w + r_top p~(r')) equals the last claim of sum-check 2;
and sum_col t[col] G_col = sum_row eq(r_row, row) C_row.
"""
import hashlib
import struct

from .bn254 import R, g1_eq, g1_msm
from . import r1cs

DOMAIN = b"zkvc-spartan-v1"


# ------------------------------------------------------------------ transcript
def fr_bytes(v):
    return int(v % R).to_bytes(32, "little")


def g1_bytes(p):
    if p is None:
        return bytes(64)
    return int(p[0]).to_bytes(32, "little") + int(p[1]).to_bytes(32, "little")


class Transcript:
    """SHA-256 chain: state' = H(state || label || data); a challenge is
    (H(state || label || 00) || H(state || label || 01)) read as a 512-bit
    little-endian integer mod r, after which state' = H(state || label || 02)."""

    def __init__(self):
        self.state = hashlib.sha256(DOMAIN).digest()

    def absorb(self, label, data):
        self.state = hashlib.sha256(self.state + label + data).digest()

    def challenge(self, label):
        lo = hashlib.sha256(self.state + label + b"\x00").digest()
        hi = hashlib.sha256(self.state + label + b"\x01").digest()
        self.state = hashlib.sha256(self.state + label + b"\x02").digest()
        return int.from_bytes(lo + hi, "little") % R


# ------------------------------------------------------------------ multilinear helpers
def eq_eval(r, bits_of):
    """eq(r, b) for the bit vector b given as an int (bit k = coordinate k)."""
    acc = 1
    for k, rk in enumerate(r):
        acc = acc * (rk if (bits_of >> k) & 1 else (1 - rk)) % R
    return acc


def eq_table(r):
    """[eq(r, i) for i < 2^len(r)]."""
    return [eq_eval(r, i) for i in range(1 << len(r))]


def mle_eval(f, r):
    """f~(r) for len(f) = 2^len(r), by the definition."""
    assert len(f) == 1 << len(r)
    return sum(v * eq_eval(r, i) for i, v in enumerate(f)) % R


def fold(f, c):
    """Binds the least significant variable to c."""
    return [(f[2 * i] + c * (f[2 * i + 1] - f[2 * i])) % R for i in range(len(f) // 2)]


def interpolate(vals, x):
    """Value at x of the polynomial of degree < len(vals) with vals[t] at t = 0, 1, ..."""
    n = len(vals)
    acc = 0
    for i in range(n):
        num, den = 1, 1
        for j in range(n):
            if j != i:
                num = num * (x - j) % R
                den = den * (i - j) % R
        acc += vals[i] * num * pow(den, -1, R)
    return acc % R


def log2_ceil(v):
    k = 0
    while (1 << k) < v:
        k += 1
    return k


# ------------------------------------------------------------------ instance layout
class Instance:
    """Sizes and layout of the Spartan instance of one matmul circuit."""

    def __init__(self, s, kind, z=None):
        self.s, self.kind, self.z = s, kind, z
        self.m = r1cs.num_constraints(s, kind)
        self.ell = r1cs.num_public(s)
        self.nv = r1cs.num_vars(s, kind)
        self.nw = self.nv - self.ell - 1
        self.sx = max(1, log2_ceil(self.m))
        self.sw = max(1, log2_ceil(self.nw), log2_ceil(self.ell + 1))
        self.sy = self.sw + 1
        self.half = 1 << self.sw
        self.col_bits = (self.sw + 1) // 2
        self.row_bits = self.sw - self.col_bits
        self.cols = 1 << self.col_bits
        self.rows = 1 << self.row_bits
        self.zp = r1cs.z_powers(s, z) if kind in r1cs.CRPC_KINDS else None

    def column(self, v):
        """Position of variable v in z."""
        return v - (self.ell + 1) if v > self.ell else self.half + v

    def z_vector(self, a):
        z = [0] * (1 << self.sy)
        for j in range(self.nw):
            z[j] = a[self.ell + 1 + j]
        for t in range(self.ell + 1):
            z[self.half + t] = a[t]
        return z

    def constraint(self, c):
        return r1cs.row(self.s, self.kind, c, self.zp)

    def header(self):
        s = self.s
        return struct.pack("<4I", s.a, s.n, s.b, self.kind) + fr_bytes(self.z or 0)


def io_bytes(X, Y):
    """The statement's public values as bytes: X as int8, then Y as little-endian int32, row-major."""
    return b"".join(struct.pack("<b", v) for row in X for v in row) + \
        b"".join(struct.pack("<i", v) for row in Y for v in row)


def _start(inst, X, Y, comms):
    tr = Transcript()
    tr.absorb(b"shape", inst.header())
    tr.absorb(b"io", io_bytes(X, Y))
    tr.absorb(b"comm", b"".join(g1_bytes(c) for c in comms))
    return tr


def commit_rows(inst, w, gens):
    """Pedersen commitment of every row of the witness matrix."""
    assert len(gens) == inst.cols
    return [g1_msm(gens, w[i * inst.cols:(i + 1) * inst.cols]) for i in range(inst.rows)]


def m_vector(inst, rx, ra, rb, rc):
    """M(y) for every y < 2^sy, from the constraint rows."""
    ex = eq_table(rx)
    M = [0] * (1 << inst.sy)
    for c in range(inst.m):
        A, B, C = inst.constraint(c)
        for coef_w, row in ((ra, A), (rb, B), (rc, C)):
            for v, val in row.items():
                y = inst.column(v)
                M[y] = (M[y] + ex[c] * coef_w % R * val) % R
    return M


def prove(inst, X, W, gens, commitments=None):
    """Spartan proof for Y = X W: dict of commitments, sum-check messages,
    vA, vB, vC and the opening vector t; also returns Y.

    commitments: optional precomputed row commitments (for sizes where the
    oracle's double-and-add would take too long, computed by the caller
    from the oracle's own arithmetic, e.g. by the discrete-log identity)."""
    s, kind = inst.s, inst.kind
    a, Y = r1cs.assignment(s, kind, X, W, inst.z)
    z = inst.z_vector(a)
    w = z[:inst.half]
    comms = commitments if commitments is not None else commit_rows(inst, w, gens)
    tr = _start(inst, X, Y, comms)
    tau = [tr.challenge(b"tau") for _ in range(inst.sx)]
    # sum-check 1
    size = 1 << inst.sx
    E = eq_table(tau)
    Az, Bz, Cz = [0] * size, [0] * size, [0] * size
    for c in range(inst.m):
        A, B, C = inst.constraint(c)
        Az[c], Bz[c], Cz[c] = r1cs.dot(A, a), r1cs.dot(B, a), r1cs.dot(C, a)
    sc1, rx = [], []
    for _ in range(inst.sx):
        g = [0, 0, 0, 0]
        for i in range(len(E) // 2):
            for t in range(4):
                e = E[2 * i] + t * (E[2 * i + 1] - E[2 * i])
                av = Az[2 * i] + t * (Az[2 * i + 1] - Az[2 * i])
                bv = Bz[2 * i] + t * (Bz[2 * i + 1] - Bz[2 * i])
                cv = Cz[2 * i] + t * (Cz[2 * i + 1] - Cz[2 * i])
                g[t] = (g[t] + e * (av * bv - cv)) % R
        sc1.append(g)
        tr.absorb(b"sc1", b"".join(fr_bytes(v) for v in g))
        r = tr.challenge(b"r1")
        rx.append(r)
        E, Az, Bz, Cz = fold(E, r), fold(Az, r), fold(Bz, r), fold(Cz, r)
    va, vb, vc = Az[0], Bz[0], Cz[0]
    tr.absorb(b"vabc", fr_bytes(va) + fr_bytes(vb) + fr_bytes(vc))
    ra, rb, rc = tr.challenge(b"ra"), tr.challenge(b"rb"), tr.challenge(b"rc")
    # sum-check 2
    M = m_vector(inst, rx, ra, rb, rc)
    Z = list(z)
    sc2, ry = [], []
    for _ in range(inst.sy):
        g = [0, 0, 0]
        for i in range(len(M) // 2):
            for t in range(3):
                mv = M[2 * i] + t * (M[2 * i + 1] - M[2 * i])
                zv = Z[2 * i] + t * (Z[2 * i + 1] - Z[2 * i])
                g[t] = (g[t] + mv * zv) % R
        sc2.append(g)
        tr.absorb(b"sc2", b"".join(fr_bytes(v) for v in g))
        r = tr.challenge(b"r2")
        ry.append(r)
        M, Z = fold(M, r), fold(Z, r)
    # opening of the witness extension at r_y without its top coordinate
    rp = ry[:inst.sw]
    er = eq_table(rp[inst.col_bits:])
    t = [sum(er[i] * w[i * inst.cols + col] for i in range(inst.rows)) % R for col in range(inst.cols)]
    return {"comms": comms, "sc1": sc1, "vabc": (va, vb, vc), "sc2": sc2, "t": t}, Y


def matrix_eval(inst, rx, ry, ra, rb, rc):
    """M~(r_y) = sum over the nonzero entries of eq(r_x, x) eq(r_y, y) (weighted entry)."""
    acc = 0
    for c in range(inst.m):
        ex = eq_eval(rx, c)
        A, B, C = inst.constraint(c)
        for coef_w, row in ((ra, A), (rb, B), (rc, C)):
            for v, val in row.items():
                acc += ex * coef_w % R * val % R * eq_eval(ry, inst.column(v))
    return acc % R


def verify(inst, X, Y, proof, gens):
    """True iff the proof is valid for the public X and Y."""
    s = inst.s
    if len(X) != s.a or len(Y) != s.a or any(len(r) != s.n for r in X) or any(len(r) != s.b for r in Y):
        return False
    if len(proof["comms"]) != inst.rows or len(proof["t"]) != inst.cols:
        return False
    if len(proof["sc1"]) != inst.sx or len(proof["sc2"]) != inst.sy:
        return False
    pub = [1] + [X[i][k] % R for i in range(s.a) for k in range(s.n)] + \
          [Y[i][j] % R for i in range(s.a) for j in range(s.b)]
    tr = _start(inst, X, Y, proof["comms"])
    tau = [tr.challenge(b"tau") for _ in range(inst.sx)]
    claim, rx = 0, []
    for g in proof["sc1"]:
        if len(g) != 4 or (g[0] + g[1]) % R != claim:
            return False
        tr.absorb(b"sc1", b"".join(fr_bytes(v) for v in g))
        r = tr.challenge(b"r1")
        rx.append(r)
        claim = interpolate(g, r)
    va, vb, vc = proof["vabc"]
    if claim != _eq_points(tau, rx) * (va * vb - vc) % R:
        return False
    tr.absorb(b"vabc", fr_bytes(va) + fr_bytes(vb) + fr_bytes(vc))
    ra, rb, rc = tr.challenge(b"ra"), tr.challenge(b"rb"), tr.challenge(b"rc")
    claim, ry = (ra * va + rb * vb + rc * vc) % R, []
    for g in proof["sc2"]:
        if len(g) != 3 or (g[0] + g[1]) % R != claim:
            return False
        tr.absorb(b"sc2", b"".join(fr_bytes(v) for v in g))
        r = tr.challenge(b"r2")
        ry.append(r)
        claim = interpolate(g, r)
    rp, rtop = ry[:inst.sw], ry[inst.sw]
    t = proof["t"]
    ec = eq_table(rp[:inst.col_bits])
    v_w = sum(tc * e for tc, e in zip(t, ec)) % R
    p_eval = sum(v * eq_eval(rp, j) for j, v in enumerate(pub)) % R
    z_eval = ((1 - rtop) * v_w + rtop * p_eval) % R
    if claim != matrix_eval(inst, rx, ry, ra, rb, rc) * z_eval % R:
        return False
    er = eq_table(rp[inst.col_bits:])
    lhs = g1_msm(gens, [v % R for v in t])
    rhs = g1_msm(proof["comms"], er)
    return g1_eq(lhs, rhs)


def _eq_points(r, x):
    """eq(r, x) for two field-element vectors (the extension of eq to all points)."""
    acc = 1
    for rk, xk in zip(r, x):
        acc = acc * (rk * xk + (1 - rk) * (1 - xk)) % R
    return acc



def proof_bytes(proof):
    """The proof's byte encoding: commitments (64 bytes each), sum-check 1
    values, vA vB vC, sum-check 2 values, opening values (32 bytes each)."""
    out = b"".join(g1_bytes(c) for c in proof["comms"])
    out += b"".join(fr_bytes(v) for g in proof["sc1"] for v in g)
    out += b"".join(fr_bytes(v) for v in proof["vabc"])
    out += b"".join(fr_bytes(v) for g in proof["sc2"] for v in g)
    out += b"".join(fr_bytes(v) for v in proof["t"])
    return out


def proof_from_bytes(inst, data):
    """Inverse of proof_bytes for the instance's sizes (None if the length is wrong)."""
    need = inst.rows * 64 + (4 * inst.sx + 3 + 3 * inst.sy + inst.cols) * 32
    if len(data) != need:
        return None
    pts = []
    for i in range(inst.rows):
        x = int.from_bytes(data[64 * i:64 * i + 32], "little")
        y = int.from_bytes(data[64 * i + 32:64 * i + 64], "little")
        pts.append(None if x == 0 and y == 0 else (x, y))
    off = inst.rows * 64
    vals = [int.from_bytes(data[off + 32 * k:off + 32 * k + 32], "little") for k in range((len(data) - off) // 32)]
    sc1 = [vals[4 * j:4 * j + 4] for j in range(inst.sx)]
    p = 4 * inst.sx
    vabc = tuple(vals[p:p + 3])
    p += 3
    sc2 = [vals[p + 3 * j:p + 3 * j + 3] for j in range(inst.sy)]
    p += 3 * inst.sy
    return {"comms": pts, "sc1": sc1, "vabc": vabc, "sc2": sc2, "t": vals[p:p + inst.cols]}
