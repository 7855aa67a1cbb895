"""Byte encodings of proofs and verification keys, for the CPU oracle.

TEST INFRASTRUCTURE ONLY (see oracle/bn254.py).

These layouts are the library's ABI formats; this is an independent
implementation used to cross-check proofs and keys in both directions.

  field element   32 bytes, little-endian canonical integer (< modulus)
  G1 point        x || y  (64 bytes); the point at infinity is all zeros
  G2 point        x.c0 || x.c1 || y.c0 || y.c1  (128 bytes), x = c0 + c1 i;
                  infinity is all zeros
  proof           A (G1) || B (G2) || C (G1) = 256 bytes
  vk blob         magic "ZKVC-VK1" (8 bytes)
                  u32 version (=1), u32 a, u32 n, u32 b, u32 kind, u32 log2 N
                  z (32 bytes; zero for the plain circuit)
                  alpha1 (G1), beta2 (G2), gamma2 (G2), delta2 (G2)
                  u64 count (= l + 1)
                  IC_0 .. IC_l (G1 each)
"""
import struct

from .r1cs import Shape

VK_MAGIC = b"ZKVC-VK1"
VK_VERSION = 1


def fe_bytes(v):
    return int(v).to_bytes(32, "little")


def fe_from(b):
    return int.from_bytes(b[:32], "little")


def g1_bytes(pt):
    if pt is None:
        return bytes(64)
    return fe_bytes(pt[0]) + fe_bytes(pt[1])


def g1_from(b):
    x, y = fe_from(b[0:32]), fe_from(b[32:64])
    return None if x == 0 and y == 0 else (x, y)


def g2_bytes(pt):
    if pt is None:
        return bytes(128)
    (x0, x1), (y0, y1) = pt
    return fe_bytes(x0) + fe_bytes(x1) + fe_bytes(y0) + fe_bytes(y1)


def g2_from(b):
    v = [fe_from(b[32 * k:32 * k + 32]) for k in range(4)]
    return None if not any(v) else ((v[0], v[1]), (v[2], v[3]))


def proof_bytes(proof):
    return g1_bytes(proof[0]) + g2_bytes(proof[1]) + g1_bytes(proof[2])


def proof_from(b):
    return (g1_from(b[0:64]), g2_from(b[64:192]), g1_from(b[192:256]))


def vk_blob(vk):
    s = vk["shape"]
    log_n = vk["N"].bit_length() - 1
    out = VK_MAGIC + struct.pack("<6I", VK_VERSION, s.a, s.n, s.b, vk["kind"], log_n)
    out += fe_bytes(vk["z"] or 0)
    out += g1_bytes(vk["alpha1"]) + g2_bytes(vk["beta2"]) + g2_bytes(vk["gamma2"]) + g2_bytes(vk["delta2"])
    out += struct.pack("<Q", len(vk["IC"]))
    out += b"".join(g1_bytes(p) for p in vk["IC"])
    return out


def vk_from_blob(blob):
    if blob[:8] != VK_MAGIC:
        raise ValueError("bad vk magic")
    version, a, n, b, kind, log_n = struct.unpack("<6I", blob[8:32])
    if version != VK_VERSION:
        raise ValueError("unsupported vk version")
    off = 32
    z = fe_from(blob[off:off + 32]); off += 32
    alpha1 = g1_from(blob[off:off + 64]); off += 64
    beta2 = g2_from(blob[off:off + 128]); off += 128
    gamma2 = g2_from(blob[off:off + 128]); off += 128
    delta2 = g2_from(blob[off:off + 128]); off += 128
    (count,) = struct.unpack("<Q", blob[off:off + 8]); off += 8
    if len(blob) != off + 64 * count:
        raise ValueError("bad vk length")
    ic = [g1_from(blob[off + 64 * k: off + 64 * k + 64]) for k in range(count)]
    return {"shape": Shape(a, n, b), "kind": kind, "N": 1 << log_n, "z": z or None,
            "alpha1": alpha1, "beta2": beta2, "gamma2": gamma2, "delta2": delta2, "IC": ic}
