"""ctypes binding for libzkvc.so: argument marshalling only.

Every computation runs in the library's HIP kernels (or, for verification and
the prover's serial tails, in its host C++).  PyTorch is used by callers for
device memory and streams; this module only passes pointers and sizes.  If
the library is missing, loading fails loudly: there is no fallback path.
"""
import ctypes
import os
import struct

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libzkvc.so")

OK, EINVAL, ENOMEM, EDEVICE, EFORMAT = 0, -1, -2, -3, -4
PLAIN, CRPC_PSQ, PLAIN_ADD, PLAIN_PSQ, CRPC = 0, 1, 2, 3, 4
NTT_INVERSE, NTT_COSET, LAYOUT_MONT = 1, 2, 4
TUNE_MSM_G1, TUNE_MSM_G2, TUNE_NTT = 1, 2, 4
Q_A, Q_B1, Q_B2, Q_L, Q_H, Q_CONST = 0, 1, 2, 3, 4, 5
FQ, FR = 0, 1
OP_ADD, OP_SUB, OP_MUL, OP_SQR, OP_INV, OP_TO_MONT, OP_FROM_MONT = range(7)


class ZkvcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"zkvc error {code}: {msg}")
        self.code = code


class Fr(ctypes.Structure):
    _fields_ = [("l", ctypes.c_uint32 * 8)]


class G1(ctypes.Structure):
    _fields_ = [("x", ctypes.c_uint32 * 8), ("y", ctypes.c_uint32 * 8)]


class G2(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_uint32 * 8), ("x1", ctypes.c_uint32 * 8),
                ("y0", ctypes.c_uint32 * 8), ("y1", ctypes.c_uint32 * 8)]


class Proof(ctypes.Structure):
    _fields_ = [("A", G1), ("B", G2), ("C", G1)]


class Shape(ctypes.Structure):
    _fields_ = [("a", ctypes.c_uint32), ("n", ctypes.c_uint32), ("b", ctypes.c_uint32),
                ("kind", ctypes.c_uint32)]


class PkInfo(ctypes.Structure):
    _fields_ = [("a", ctypes.c_uint32), ("n", ctypes.c_uint32), ("b", ctypes.c_uint32),
                ("kind", ctypes.c_uint32), ("log_n", ctypes.c_uint32),
                ("num_vars", ctypes.c_uint64), ("num_public", ctypes.c_uint64),
                ("a_query", ctypes.c_uint64), ("b_query", ctypes.c_uint64),
                ("l_query", ctypes.c_uint64), ("h_query", ctypes.c_uint64),
                ("device_bytes", ctypes.c_uint64), ("prove_bytes", ctypes.c_uint64)]


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_uint64), ("total_ms", ctypes.c_double),
                ("work", ctypes.c_double)]


class ProveJob(ctypes.Structure):
    _fields_ = [("pk", ctypes.c_void_p), ("X", ctypes.c_void_p), ("W", ctypes.c_void_p), ("r", Fr), ("s", Fr),
                ("Y_out", ctypes.c_void_p), ("proof_out", ctypes.POINTER(Proof))]


class ServerConfig(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_uint32), ("memory_budget", ctypes.c_uint64)]


class ServerResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("batch_size", ctypes.c_uint32), ("queue_ms", ctypes.c_double),
                ("latency_ms", ctypes.c_double)]


class ValuPeak(ctypes.Structure):
    _fields_ = [("mads", ctypes.c_double), ("ms", ctypes.c_double), ("mad_per_s", ctypes.c_double),
                ("clock_ghz", ctypes.c_double), ("lane_ops_per_cu_clk", ctypes.c_double),
                ("compute_units", ctypes.c_uint32)]


class SpartanInfo(ctypes.Structure):
    _fields_ = [("constraints", ctypes.c_uint64), ("sx", ctypes.c_uint32), ("sy", ctypes.c_uint32),
                ("rows", ctypes.c_uint32), ("cols", ctypes.c_uint32), ("proof_bytes", ctypes.c_uint64)]


class ProveStats(ctypes.Structure):
    _fields_ = [("witness_ms", ctypes.c_float), ("ntt_ms", ctypes.c_float), ("msm_ms", ctypes.c_float),
                ("host_ms", ctypes.c_float), ("total_ms", ctypes.c_float)]


_lib = None

_VP = ctypes.c_void_p
_SIGS = {
    "zkvc_setup": (ctypes.c_int, [ctypes.POINTER(Shape), ctypes.POINTER(Fr), ctypes.POINTER(Fr),
                                  ctypes.POINTER(_VP), ctypes.c_char_p, ctypes.POINTER(ctypes.c_size_t), _VP]),
    "zkvc_pk_free": (ctypes.c_int, [_VP]),
    "zkvc_prove": (ctypes.c_int, [_VP, _VP, _VP, ctypes.POINTER(Fr), ctypes.POINTER(Fr), _VP,
                                  ctypes.POINTER(Proof), _VP]),
    "zkvc_prove_device": (ctypes.c_int, [_VP, _VP, _VP, ctypes.POINTER(Fr), ctypes.POINTER(Fr), _VP,
                                         ctypes.POINTER(Proof), _VP]),
    "zkvc_prove_batch": (ctypes.c_int, [ctypes.POINTER(ProveJob), ctypes.c_size_t, _VP]),
    "zkvc_server_create": (ctypes.c_int, [ctypes.POINTER(ServerConfig), ctypes.POINTER(_VP)]),
    "zkvc_server_submit": (ctypes.c_int, [_VP, ctypes.POINTER(ProveJob), ctypes.POINTER(ctypes.c_uint64)]),
    "zkvc_server_wait": (ctypes.c_int, [_VP, ctypes.c_uint64, ctypes.POINTER(ServerResult)]),
    "zkvc_server_destroy": (ctypes.c_int, [_VP]),
    "zkvc_autotune": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, _VP]),
    "zkvc_tune_export": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_size_t)]),
    "zkvc_tune_import": (ctypes.c_int, [ctypes.c_char_p]),
    "zkvc_set_graphs": (ctypes.c_int, [ctypes.c_int]),
    "zkvc_profile_select": (ctypes.c_int, [ctypes.c_char_p]),
    "zkvc_verify": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_size_t, _VP, _VP, ctypes.POINTER(Proof)]),
    "zkvc_ntt_fr": (ctypes.c_int, [_VP, ctypes.c_uint32, ctypes.c_uint32, _VP]),
    "zkvc_msm_g1": (ctypes.c_int, [_VP, _VP, ctypes.c_size_t, ctypes.c_uint32, ctypes.POINTER(G1), _VP]),
    "zkvc_msm_g2": (ctypes.c_int, [_VP, _VP, ctypes.c_size_t, ctypes.c_uint32, ctypes.POINTER(G2), _VP]),
    "zkvc_msm_g1_noalloc": (ctypes.c_int, [_VP, _VP, ctypes.c_size_t, ctypes.c_uint32, ctypes.POINTER(G1), _VP]),
    "zkvc_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "zkvc_fixed_base_g1": (ctypes.c_int, [_VP, ctypes.c_size_t, _VP, ctypes.c_uint32, _VP]),
    "zkvc_fixed_base_g2": (ctypes.c_int, [_VP, ctypes.c_size_t, _VP, ctypes.c_uint32, _VP]),
    "zkvc_pk_info": (ctypes.c_int, [_VP, ctypes.POINTER(PkInfo)]),
    "zkvc_pk_export": (ctypes.c_int, [_VP, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, _VP]),
    "zkvc_pk_last_stats": (ctypes.c_int, [_VP, ctypes.POINTER(ProveStats)]),
    "zkvc_field_op": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32, _VP, _VP, _VP, ctypes.c_size_t, _VP]),
    "zkvc_valu_peak": (ctypes.c_int, [ctypes.c_uint32, ctypes.POINTER(ValuPeak), _VP]),
    "zkvc_spartan_info": (ctypes.c_int, [ctypes.POINTER(Shape), ctypes.POINTER(SpartanInfo)]),
    "zkvc_spartan_setup": (ctypes.c_int, [ctypes.POINTER(Shape), ctypes.POINTER(Fr), _VP, ctypes.c_size_t,
                                          ctypes.POINTER(_VP), _VP]),
    "zkvc_spartan_key_free": (ctypes.c_int, [_VP]),
    "zkvc_spartan_prove": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, ctypes.c_size_t, _VP]),
    "zkvc_spartan_verify": (ctypes.c_int, [ctypes.POINTER(Shape), ctypes.POINTER(Fr), _VP, ctypes.c_size_t, _VP, _VP,
                                           _VP, ctypes.c_size_t]),
    "zkvc_profile_begin": (ctypes.c_int, []),
    "zkvc_profile_read": (ctypes.c_int, [ctypes.POINTER(KernelStat), ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
}

EXPORTS = tuple(_SIGS)


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2504_12217_amd.build`")
        try:
            # torch brings its own HIP runtime; loading it first makes the
            # library bind to that same runtime, so that torch's device
            # pointers and streams are valid here whatever the import order
            import torch  # noqa: F401
        except ImportError:
            pass
        _lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(_lib, name)
            f.restype = res
            f.argtypes = args
    return _lib


def _check(code):
    if code < 0:
        msg = lib().zkvc_strerror(code)
        raise ZkvcError(code, msg.decode() if msg else "")
    return code


def _ptr(t):
    """Device pointer of a torch tensor (or an int address)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return stream if isinstance(stream, int) else stream.cuda_stream


# -------------------------------------------------------------------- value marshalling
def fr(v):
    out = Fr()
    for k in range(8):
        out.l[k] = (int(v) >> (32 * k)) & 0xFFFFFFFF
    return out


def words_to_int(ws):
    return sum(int(w) << (32 * k) for k, w in enumerate(ws))


def g1_to_tuple(p):
    x, y = words_to_int(p.x), words_to_int(p.y)
    return None if x == 0 and y == 0 else (x, y)


def g2_to_tuple(p):
    v = [words_to_int(p.x0), words_to_int(p.x1), words_to_int(p.y0), words_to_int(p.y1)]
    return None if not any(v) else ((v[0], v[1]), (v[2], v[3]))


def proof_to_tuple(p):
    return (g1_to_tuple(p.A), g2_to_tuple(p.B), g1_to_tuple(p.C))


def proof_bytes(p):
    return bytes(p)


def proof_from_bytes(b):
    p = Proof()
    ctypes.memmove(ctypes.addressof(p), bytes(b), ctypes.sizeof(Proof))
    return p


# -------------------------------------------------------------------- kernels
def ntt_fr(data, log_n, flags=0, stream=None):
    _check(lib().zkvc_ntt_fr(_ptr(data), log_n, flags, _stream(stream)))


def msm_g1(points, scalars, n, flags=0, stream=None):
    out = G1()
    _check(lib().zkvc_msm_g1(_ptr(points), _ptr(scalars), n, flags, ctypes.byref(out), _stream(stream)))
    return g1_to_tuple(out)


def msm_g1_noalloc(points, scalars, n, flags=0, stream=None):
    """zkvc_msm_g1 on the library's fixed scratch (no allocation); n <= 65536."""
    out = G1()
    _check(lib().zkvc_msm_g1_noalloc(_ptr(points), _ptr(scalars), n, flags, ctypes.byref(out), _stream(stream)))
    return g1_to_tuple(out)


def msm_g2(points, scalars, n, flags=0, stream=None):
    out = G2()
    _check(lib().zkvc_msm_g2(_ptr(points), _ptr(scalars), n, flags, ctypes.byref(out), _stream(stream)))
    return g2_to_tuple(out)


def fixed_base_g1(scalars, n, points_out, flags=0, stream=None):
    _check(lib().zkvc_fixed_base_g1(_ptr(scalars), n, _ptr(points_out), flags, _stream(stream)))


def fixed_base_g2(scalars, n, points_out, flags=0, stream=None):
    _check(lib().zkvc_fixed_base_g2(_ptr(scalars), n, _ptr(points_out), flags, _stream(stream)))


def field_op(field, op, a, b, out, n, stream=None):
    _check(lib().zkvc_field_op(field, op, _ptr(a), _ptr(b), _ptr(out), n, _stream(stream)))


def autotune(what=TUNE_MSM_G1 | TUNE_MSM_G2 | TUNE_NTT, min_log=10, max_log=16, stream=None):
    """Tune on the device; returns the number of settings chosen."""
    return _check(lib().zkvc_autotune(what, min_log, max_log, _stream(stream)))


def tune_export():
    n = ctypes.c_size_t(0)
    _check(lib().zkvc_tune_export(None, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value)
    _check(lib().zkvc_tune_export(buf, ctypes.byref(n)))
    return buf.value.decode()


def tune_import(text):
    _check(lib().zkvc_tune_import(text.encode()))


def set_graphs(enable):
    """Turn graph capture and replay of repeated proof compositions on or off
    (off by default); returns the previous setting."""
    return lib().zkvc_set_graphs(1 if enable else 0)


def valu_peak(iters=4096, stream=None):
    """The device's measured v_mad_u64_u32 rate (zkvc_valu_peak): a dict of its fields."""
    out = ValuPeak()
    _check(lib().zkvc_valu_peak(iters, ctypes.byref(out), _stream(stream)))
    return {k: getattr(out, k) for k, _ in ValuPeak._fields_}


def profile_begin():
    """Start recording HIP events around the library's instrumented launches."""
    _check(lib().zkvc_profile_begin())


def profile_select(kernels=None):
    """Record only the launches of the named kernels (a name or a list of names; None: all)."""
    if isinstance(kernels, (list, tuple, set)):
        kernels = ",".join(sorted(kernels))
    _check(lib().zkvc_profile_select(kernels.encode() if kernels else None))


def profile_read():
    """Stop recording; {kernel: (launches, total_ms, work_units)}."""
    buf = (KernelStat * 128)()
    cnt = ctypes.c_int(0)
    _check(lib().zkvc_profile_read(buf, 128, ctypes.byref(cnt)))
    return {buf[k].name.decode(): (buf[k].launches, buf[k].total_ms, buf[k].work) for k in range(min(cnt.value, 128))}


# -------------------------------------------------------------------- Groth16
class ProvingKey:
    """Owns a device-resident proving key; frees it on close() or garbage collection."""

    def __init__(self, handle, vk):
        self.handle = handle
        self.vk = vk

    def close(self):
        if self.handle:
            lib().zkvc_pk_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        out = PkInfo()
        _check(lib().zkvc_pk_info(self.handle, ctypes.byref(out)))
        return out

    def last_stats(self):
        out = ProveStats()
        _check(lib().zkvc_pk_last_stats(self.handle, ctypes.byref(out)))
        return out

    def export(self, query, start, count):
        """Canonical affine points of a proving-key query (list of tuples)."""
        if query == Q_CONST:
            buf = (ctypes.c_uint8 * (3 * 64 + 2 * 128))()
            _check(lib().zkvc_pk_export(self.handle, query, 0, 0, ctypes.cast(buf, _VP)))
            raw = bytes(buf)
            g1s = [G1.from_buffer_copy(raw[64 * k:64 * k + 64]) for k in range(3)]
            g2s = [G2.from_buffer_copy(raw[192 + 128 * k:192 + 128 * k + 128]) for k in range(2)]
            return [g1_to_tuple(p) for p in g1s] + [g2_to_tuple(p) for p in g2s]
        width = 128 if query == Q_B2 else 64
        buf = (ctypes.c_uint8 * (width * max(count, 1)))()
        _check(lib().zkvc_pk_export(self.handle, query, start, count, ctypes.cast(buf, _VP)))
        raw = bytes(buf)
        if width == 128:
            return [g2_to_tuple(G2.from_buffer_copy(raw[128 * k:128 * k + 128])) for k in range(count)]
        return [g1_to_tuple(G1.from_buffer_copy(raw[64 * k:64 * k + 64])) for k in range(count)]


def setup(a, n, b, kind, toxic, z=None, stream=None):
    """Key generation; toxic = (tau, alpha, beta, gamma, delta) as ints.  Returns ProvingKey."""
    shape = Shape(a, n, b, kind)
    tox = (Fr * 5)(*[fr(v) for v in toxic])
    zz = fr(z) if z is not None else None
    handle = _VP()
    need = ctypes.c_size_t(0)
    _check(lib().zkvc_setup(ctypes.byref(shape), tox, ctypes.byref(zz) if zz is not None else None,
                            None, None, ctypes.byref(need), _stream(stream)))
    buf = ctypes.create_string_buffer(need.value)
    cap = ctypes.c_size_t(need.value)
    _check(lib().zkvc_setup(ctypes.byref(shape), tox, ctypes.byref(zz) if zz is not None else None,
                            ctypes.byref(handle), buf, ctypes.byref(cap), _stream(stream)))
    return ProvingKey(handle.value, buf.raw[:cap.value])


def prove(pk, X, W, r, s, stream=None):
    """X int8 [a, n], W int8 [n, b] numpy arrays; returns (Y int32 [a, b], Proof)."""
    info = pk.info()
    X = np.ascontiguousarray(X, dtype=np.int8)
    W = np.ascontiguousarray(W, dtype=np.int8)
    if X.shape != (info.a, info.n) or W.shape != (info.n, info.b):
        raise ValueError("X or W does not match the proving key's shape")
    Y = np.zeros((info.a, info.b), dtype=np.int32)
    out = Proof()
    rr, ss = fr(r), fr(s)
    _check(lib().zkvc_prove(pk.handle, X.ctypes.data, W.ctypes.data, ctypes.byref(rr), ctypes.byref(ss),
                            Y.ctypes.data, ctypes.byref(out), _stream(stream)))
    return Y, out


def prove_device(pk, X, W, r, s, Y, stream=None):
    """X int8 [a, n], W int8 [n, b] and Y int32 [a, b] contiguous device tensors
    on the key's device; writes Y and returns the Proof."""
    info = pk.info()
    if tuple(X.shape) != (info.a, info.n) or tuple(W.shape) != (info.n, info.b) or tuple(Y.shape) != (info.a, info.b):
        raise ValueError("X, W or Y does not match the proving key's shape")
    for t, dt in ((X, "int8"), (W, "int8"), (Y, "int32")):
        if str(t.dtype) != "torch." + dt or not t.is_contiguous():
            raise ValueError(f"expected a contiguous {dt} tensor")
    out = Proof()
    rr, ss = fr(r), fr(s)
    _check(lib().zkvc_prove_device(pk.handle, _ptr(X), _ptr(W), ctypes.byref(rr), ctypes.byref(ss), _ptr(Y),
                                   ctypes.byref(out), _stream(stream)))
    return out


def prove_batch(jobs, stream=None):
    """jobs: sequence of (pk, X, W, r, s); returns [(Y, Proof)] in the same order."""
    keep = []
    arr = (ProveJob * len(jobs))()
    outs = []
    for k, (pk, X, W, r, s) in enumerate(jobs):
        info = pk.info()
        X = np.ascontiguousarray(X, dtype=np.int8)
        W = np.ascontiguousarray(W, dtype=np.int8)
        if X.shape != (info.a, info.n) or W.shape != (info.n, info.b):
            raise ValueError(f"job {k}: X or W does not match its proving key's shape")
        Y = np.zeros((info.a, info.b), dtype=np.int32)
        out = Proof()
        keep += [X, W]
        outs.append((Y, out))
        arr[k].pk = pk.handle
        arr[k].X = X.ctypes.data
        arr[k].W = W.ctypes.data
        arr[k].r = fr(r)
        arr[k].s = fr(s)
        arr[k].Y_out = Y.ctypes.data
        arr[k].proof_out = ctypes.pointer(out)
    _check(lib().zkvc_prove_batch(arr, len(jobs), _stream(stream)))
    return outs


class Server:
    """The library's proving server: submit jobs as they arrive, wait for each ticket."""

    def __init__(self, max_batch=64, memory_budget=0):
        cfg = ServerConfig(max_batch, memory_budget)
        h = _VP()
        _check(lib().zkvc_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h.value
        self._pending = {}  # ticket -> (Y, Proof, inputs kept alive)

    def submit(self, pk, X, W, r, s):
        info = pk.info()
        X = np.ascontiguousarray(X, dtype=np.int8)
        W = np.ascontiguousarray(W, dtype=np.int8)
        if X.shape != (info.a, info.n) or W.shape != (info.n, info.b):
            raise ValueError("X or W does not match the proving key's shape")
        Y = np.zeros((info.a, info.b), dtype=np.int32)
        out = Proof()
        job = ProveJob()
        job.pk = pk.handle
        job.X = X.ctypes.data
        job.W = W.ctypes.data
        job.r = fr(r)
        job.s = fr(s)
        job.Y_out = Y.ctypes.data
        job.proof_out = ctypes.pointer(out)
        t = ctypes.c_uint64(0)
        _check(lib().zkvc_server_submit(self.handle, ctypes.byref(job), ctypes.byref(t)))
        self._pending[t.value] = (Y, out)
        return t.value

    def wait(self, ticket):
        """(Y, Proof, ServerResult) of a ticket; raises ZkvcError if its batch failed."""
        res = ServerResult()
        _check(lib().zkvc_server_wait(self.handle, ticket, ctypes.byref(res)))
        Y, out = self._pending.pop(ticket)
        _check(res.status)
        return Y, out, res

    def close(self):
        if self.handle:
            _check(lib().zkvc_server_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def verify(vk, X, Y, proof):
    """1 if valid, 0 if not; raises on malformed input."""
    X = np.ascontiguousarray(X, dtype=np.int8)
    Y = np.ascontiguousarray(Y, dtype=np.int32)
    if not isinstance(proof, Proof):
        proof = proof_from_bytes(proof)
    return _check(lib().zkvc_verify(vk, len(vk), X.ctypes.data, Y.ctypes.data, ctypes.byref(proof)))


def vk_header(vk):
    """(a, n, b, kind, log_n) from a verification-key blob."""
    _, a, n, b, kind, log_n = struct.unpack("<6I", vk[8:32])
    return a, n, b, kind, log_n


# -------------------------------------------------------------------- Spartan (zkVC-S)
def spartan_info(a, n, b, kind):
    out = SpartanInfo()
    _check(lib().zkvc_spartan_info(ctypes.byref(Shape(a, n, b, kind)), ctypes.byref(out)))
    return out


def _g1_array(points):
    arr = (G1 * len(points))()
    for k, (x, y) in enumerate(points):
        for q in range(8):
            arr[k].x[q] = (int(x) >> (32 * q)) & 0xFFFFFFFF
            arr[k].y[q] = (int(y) >> (32 * q)) & 0xFFFFFFFF
    return arr


class SpartanKey:
    """A device-resident Spartan key: shape, z and the commitment generators."""

    def __init__(self, a, n, b, kind, z, gens, stream=None):
        self.shape = (a, n, b, kind)
        self.z = z
        self.gens = _g1_array(gens)
        self.info = spartan_info(a, n, b, kind)
        h = _VP()
        zz = fr(z)
        _check(lib().zkvc_spartan_setup(ctypes.byref(Shape(a, n, b, kind)), ctypes.byref(zz),
                                        ctypes.cast(self.gens, _VP), len(gens), ctypes.byref(h), _stream(stream)))
        self.handle = h.value

    def prove(self, X, W, stream=None):
        """(Y int32 [a, b], proof bytes)."""
        a, n, b, _ = self.shape
        X = np.ascontiguousarray(X, dtype=np.int8)
        W = np.ascontiguousarray(W, dtype=np.int8)
        if X.shape != (a, n) or W.shape != (n, b):
            raise ValueError("X or W does not match the key's shape")
        Y = np.zeros((a, b), dtype=np.int32)
        buf = (ctypes.c_uint8 * self.info.proof_bytes)()
        _check(lib().zkvc_spartan_prove(self.handle, X.ctypes.data, W.ctypes.data, Y.ctypes.data,
                                        ctypes.cast(buf, _VP), self.info.proof_bytes, _stream(stream)))
        return Y, bytes(buf)

    def verify(self, X, Y, proof):
        a, n, b, kind = self.shape
        X = np.ascontiguousarray(X, dtype=np.int8)
        Y = np.ascontiguousarray(Y, dtype=np.int32)
        pb = (ctypes.c_uint8 * len(proof)).from_buffer_copy(proof)
        zz = fr(self.z)
        return _check(lib().zkvc_spartan_verify(ctypes.byref(Shape(a, n, b, kind)), ctypes.byref(zz),
                                                ctypes.cast(self.gens, _VP), len(self.gens), X.ctypes.data,
                                                Y.ctypes.data, ctypes.cast(pb, _VP), len(proof)))

    def close(self):
        if self.handle:
            lib().zkvc_spartan_key_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
