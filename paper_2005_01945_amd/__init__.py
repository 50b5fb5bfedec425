"""Thin Python binding of libfhe_mi355x.so (include/fhe.h).

Argument marshalling only: every step of gate bootstrapping runs in the HIP
kernels of the library.  Functions named fhe_* mirror the C ABI one to one;
device buffers are torch tensors (their data_ptr()), streams are torch
streams.  Importing never falls back to anything: if the library is not built
the first call raises.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# FHE_LIBRARY may point at another build of the same C ABI (e.g. a variant
# under comparison); by default the in-tree build is used.
LIB_PATH = os.environ.get("FHE_LIBRARY") or os.path.join(_HERE, "libfhe_mi355x.so")

FHE_OK, FHE_EINVAL, FHE_ENOMEM, FHE_EDEVICE, FHE_EBUSY, FHE_ECANCELED, FHE_EIO = 0, -1, -2, -3, -4, -5, -6
AND, NAND, OR, NOR, XOR, XNOR, ANDNY, ANDYN, ORNY, ORYN = range(10)
MAJ, XOR3 = 10, 11  # three-input gates (fhe_bootstrap_gate3_batch, circuits)
WORDS = 501  # n + 1 words per LWE sample
# circuit kinds of fhe_circuit_shape / fhe_circuit_schedule / fhe_debug_plan
CIRCUIT_KINDS = {"add": 0, "mul": 1, "matvec": 2, "mul_tree": 3, "karatsuba": 4, "add_numberwise": 5,
                 "matmul": 6, "add_fa": 7, "add_compound": 8}


class FheError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class fhe_params(C.Structure):
    _fields_ = [("n", C.c_uint32), ("N", C.c_uint32), ("k", C.c_uint32), ("bk_l", C.c_uint32),
                ("bk_bgbit", C.c_uint32), ("ks_t", C.c_uint32), ("ks_basebit", C.c_uint32),
                ("lwe_stdev", C.c_double), ("bk_stdev", C.c_double)]


_vp = C.c_void_p
class fhe_launch_config(C.Structure):
    _fields_ = [("waves_per_gate", C.c_uint32), ("gates_per_group", C.c_uint32), ("arith", C.c_uint32)]


class fhe_launch_record(C.Structure):
    _fields_ = [("gates", C.c_uint64), ("waves_per_gate", C.c_uint32), ("gates_per_group", C.c_uint32),
                ("arith", C.c_uint32), ("reserved", C.c_uint32),
                ("blind_rotate_ms", C.c_double), ("key_switch_ms", C.c_double)]


_SIGS = {
    "fhe_default_params": (C.c_int, [C.POINTER(fhe_params)]),
    "fhe_keygen": (C.c_int, [C.POINTER(fhe_params), C.c_uint64, C.POINTER(_vp), C.POINTER(_vp)]),
    "fhe_keygen_with_keys": (C.c_int, [C.POINTER(fhe_params), C.c_uint64, _vp, _vp, C.POINTER(_vp), C.POINTER(_vp)]),
    "fhe_secret_key_free": (None, [_vp]),
    "fhe_cloud_key_free": (None, [_vp]),
    "fhe_secret_key_export": (C.c_int, [_vp, _vp, _vp]),
    "fhe_cloud_key_export": (C.c_int, [_vp, _vp, _vp]),
    "fhe_cloud_key_params": (C.c_int, [_vp, C.POINTER(fhe_params)]),
    "fhe_key_save": (C.c_int, [_vp, _vp, C.c_char_p]),
    "fhe_key_load": (C.c_int, [C.c_char_p, C.POINTER(_vp), C.POINTER(_vp)]),
    "fhe_encrypt_bits": (C.c_int, [_vp, _vp, C.c_size_t, C.c_uint64, _vp]),
    "fhe_encrypt_uint": (C.c_int, [_vp, _vp, C.c_size_t, C.c_uint32, C.c_uint64, _vp]),
    "fhe_decrypt_bits": (C.c_int, [_vp, _vp, C.c_size_t, _vp]),
    "fhe_decrypt_uint": (C.c_int, [_vp, _vp, C.c_size_t, C.c_uint32, _vp]),
    "fhe_phase": (C.c_int, [_vp, _vp, C.c_size_t, _vp]),
    "fhe_ctx_create": (C.c_int, [_vp, C.c_int, C.POINTER(_vp)]),
    "fhe_ctx_destroy": (None, [_vp]),
    "fhe_bootstrap_gate_batch": (C.c_int, [_vp, _vp, _vp, _vp, _vp, C.c_size_t, _vp]),
    "fhe_bootstrap_gate_plain": (C.c_int, [_vp, C.c_uint8, _vp, _vp, _vp, _vp]),
    "fhe_add": (C.c_int, [_vp, _vp, _vp, _vp, C.c_size_t, C.c_uint32, _vp]),
    "fhe_mul": (C.c_int, [_vp, _vp, _vp, _vp, C.c_size_t, C.c_uint32, _vp]),
    "fhe_mul_tree": (C.c_int, [_vp, _vp, _vp, _vp, C.c_size_t, C.c_uint32, _vp]),
    "fhe_add_numberwise": (C.c_int, [_vp, _vp, _vp, _vp, C.c_size_t, C.c_uint32, _vp]),
    "fhe_add_fa": (C.c_int, [_vp, _vp, _vp, _vp, C.c_size_t, C.c_uint32, _vp]),
    "fhe_bootstrap_gate3_batch": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, C.c_size_t, _vp]),
    "fhe_bootstrap_lut_batch": (C.c_int, [_vp, _vp, _vp, _vp, C.c_size_t, _vp]),
    "fhe_bootstrap_compound_batch": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, C.c_size_t, _vp]),
    "fhe_bootstrap_gate_batch_noalloc": (C.c_int, [_vp, _vp, _vp, _vp, _vp, C.c_size_t, _vp]),
    "fhe_ctx_check": (C.c_int, [_vp]),
    "fhe_add_compound": (C.c_int, [_vp, _vp, _vp, _vp, C.c_size_t, C.c_uint32, _vp]),
    "fhe_matmul": (C.c_int, [_vp, _vp, _vp, _vp, C.c_uint32, C.c_uint32, _vp]),
    "fhe_circuit_create": (C.c_int, [_vp, _vp, C.c_uint32, C.c_uint32, _vp, C.c_uint32, C.POINTER(_vp)]),
    "fhe_circuit_run": (C.c_int, [_vp, _vp, _vp, C.c_size_t, _vp]),
    "fhe_circuit_destroy": (None, [_vp]),
    "fhe_mul_karatsuba": (C.c_int, [_vp, _vp, _vp, _vp, C.c_size_t, C.c_uint32, _vp]),
    "fhe_matvec": (C.c_int, [_vp, _vp, _vp, _vp, C.c_uint32, C.c_uint32, C.c_uint32, _vp]),
    "fhe_circuit_schedule": (C.c_int, [C.c_int, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64, C.c_uint32,
                                       C.POINTER(C.c_uint64), C.c_uint32, C.POINTER(C.c_uint32)]),
    "fhe_circuit_shape": (C.c_int, [C.c_int, C.c_uint32, C.c_uint32, C.c_uint32,
                                    C.POINTER(C.c_uint64), C.POINTER(C.c_uint32), C.POINTER(C.c_uint64)]),
    "fhe_ctx_set_timing": (C.c_int, [_vp, C.c_int]),
    "fhe_ctx_set_graphs": (C.c_int, [_vp, C.c_int]),
    "fhe_ctx_autotune": (C.c_int, [_vp, C.c_uint32, C.c_uint32]),
    "fhe_ctx_timing_launches": (C.c_int, [_vp, C.POINTER(fhe_launch_record), C.c_size_t, C.POINTER(C.c_size_t)]),
    "fhe_ctx_launch_config": (C.c_int, [_vp, C.c_uint32, C.POINTER(fhe_launch_config)]),
    "fhe_ctx_set_launch_config": (C.c_int, [_vp, C.c_uint32, C.c_uint32, C.POINTER(fhe_launch_config)]),
    "fhe_ctx_timing": (C.c_int, [_vp, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                 C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
    "fhe_serve_create": (C.c_int, [_vp, C.c_size_t, C.POINTER(_vp)]),
    "fhe_serve_submit": (C.c_int, [_vp, _vp, C.POINTER(C.c_uint64)]),
    "fhe_serve_poll": (C.c_int, [_vp, C.c_uint64, C.POINTER(C.c_int), C.POINTER(C.c_double)]),
    "fhe_serve_wait": (C.c_int, [_vp, C.c_uint64, C.c_double]),
    "fhe_serve_job_times": (C.c_int, [_vp, C.c_uint64, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "fhe_serve_cancel": (C.c_int, [_vp, C.c_uint64]),
    "fhe_serve_stats": (C.c_int, [_vp, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                                  C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
    "fhe_serve_destroy": (None, [_vp]),
    "fhe_last_error": (C.c_char_p, []),
    "fhe_debug_cmux": (C.c_int, [C.c_int, C.c_int, _vp, C.c_int32, _vp]),
    "fhe_debug_valu_rate": (C.c_int, [C.c_int, C.c_int, C.POINTER(C.c_double)]),
    "fhe_debug_plan": (C.c_int, [_vp, C.c_int, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64, _vp, C.c_uint64,
                                 _vp, C.c_uint32, C.POINTER(C.c_uint64), C.POINTER(C.c_uint32)]),
    "fhe_debug_read_wires": (C.c_int, [_vp, C.c_int, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64, _vp, _vp, _vp,
                                       _vp, C.c_size_t, _vp]),
}

_lib = None


def lib():
    """The loaded C library.  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FheError(FHE_EDEVICE, f"{LIB_PATH} is not built (python -m paper_2005_01945_amd.build)")
        # torch bundles its own HIP runtime with the same soname as the system
        # one; loading torch first makes the library bind to that single copy
        # (two HIP runtimes in one process cannot share device memory).
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def _check(rc, name):
    if rc != FHE_OK:
        raise FheError(rc, f"{name}: {lib().fhe_last_error().decode()}")


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data


def _dev(t):
    """Device pointer of a contiguous torch tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("device buffers must be contiguous")
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else stream


# ---------------------------------------------------------------------------
# Same-named wrappers of the C ABI.
# ---------------------------------------------------------------------------

def fhe_default_params() -> fhe_params:
    P = fhe_params()
    _check(lib().fhe_default_params(C.byref(P)), "fhe_default_params")
    return P


class SecretKey:
    def __init__(self, handle, params):
        self.h, self.P = handle, params

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.fhe_secret_key_free(self.h)
            self.h = None

    def export(self):
        lwe = np.empty(self.P.n, np.int32)
        tlwe = np.empty(self.P.N, np.int32)
        _check(lib().fhe_secret_key_export(self.h, lwe.ctypes.data, tlwe.ctypes.data), "fhe_secret_key_export")
        return lwe, tlwe

    def encrypt_bits(self, bits, nonce=0):
        b, pb = _host(bits, np.uint8)
        out = np.empty((b.size, WORDS), np.uint32)
        _check(lib().fhe_encrypt_bits(self.h, pb, b.size, nonce, out.ctypes.data), "fhe_encrypt_bits")
        return out

    def encrypt_uint(self, values, width, nonce=0):
        v, pv = _host(np.asarray(values).reshape(-1), np.uint64)
        out = np.empty((v.size, width, WORDS), np.uint32)
        _check(lib().fhe_encrypt_uint(self.h, pv, v.size, width, nonce, out.ctypes.data), "fhe_encrypt_uint")
        return out

    def decrypt_bits(self, ct):
        c, pc = _host(np.asarray(ct).reshape(-1, WORDS), np.uint32)
        out = np.empty(c.shape[0], np.uint8)
        _check(lib().fhe_decrypt_bits(self.h, pc, c.shape[0], out.ctypes.data), "fhe_decrypt_bits")
        return out

    def decrypt_uint(self, ct, width):
        c, pc = _host(np.asarray(ct).reshape(-1, WORDS), np.uint32)
        count = c.shape[0] // width
        out = np.empty(count, np.uint64)
        _check(lib().fhe_decrypt_uint(self.h, pc, count, width, out.ctypes.data), "fhe_decrypt_uint")
        return out

    def phase(self, ct):
        c, pc = _host(np.asarray(ct).reshape(-1, WORDS), np.uint32)
        out = np.empty(c.shape[0], np.int32)
        _check(lib().fhe_phase(self.h, pc, c.shape[0], out.ctypes.data), "fhe_phase")
        return out


class CloudKey:
    def __init__(self, handle, params):
        self.h, self.P = handle, params

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.fhe_cloud_key_free(self.h)
            self.h = None

    def export(self):
        P = self.P
        bk = np.empty((P.n, 4, 2, P.N), np.uint32)
        ksk = np.empty((P.N, P.ks_t, 1 << P.ks_basebit, P.n + 1), np.uint32)
        _check(lib().fhe_cloud_key_export(self.h, bk.ctypes.data, ksk.ctypes.data), "fhe_cloud_key_export")
        return bk, ksk


def fhe_keygen(seed=0, params=None, lwe_key=None, tlwe_key=None):
    """(SecretKey, CloudKey) from the counter-based generator keyed by seed."""
    P = params if params is not None else fhe_default_params()
    sk, ck = _vp(), _vp()
    if lwe_key is None and tlwe_key is None:
        rc = lib().fhe_keygen(C.byref(P), seed, C.byref(sk), C.byref(ck))
    else:
        lk = None if lwe_key is None else np.ascontiguousarray(lwe_key, np.int32)
        tk = None if tlwe_key is None else np.ascontiguousarray(tlwe_key, np.int32)
        rc = lib().fhe_keygen_with_keys(C.byref(P), seed, None if lk is None else lk.ctypes.data,
                                        None if tk is None else tk.ctypes.data, C.byref(sk), C.byref(ck))
    _check(rc, "fhe_keygen")
    return SecretKey(sk.value, P), CloudKey(ck.value, P)


def fhe_key_save(sk, ck, path):
    _check(lib().fhe_key_save(sk.h if sk else None, ck.h if ck else None, path.encode()), "fhe_key_save")


def fhe_key_load(path):
    sk, ck = _vp(), _vp()
    _check(lib().fhe_key_load(path.encode(), C.byref(sk), C.byref(ck)), "fhe_key_load")
    P = fhe_default_params()
    if ck.value:
        _check(lib().fhe_cloud_key_params(ck.value, C.byref(P)), "fhe_cloud_key_params")
    return (SecretKey(sk.value, P) if sk.value else None), (CloudKey(ck.value, P) if ck.value else None)


class Context:
    """Device-resident keys on one GPU (fhe_ctx)."""

    def __init__(self, cloud_key, device=0):
        h = _vp()
        _check(lib().fhe_ctx_create(cloud_key.h, device, C.byref(h)), "fhe_ctx_create")
        self.h, self.device = h.value, device

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.fhe_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


def fhe_bootstrap_gate_batch(ctx, ops, in0, in1, out, count=None, stream=None):
    count = ops.numel() if count is None else count
    _check(lib().fhe_bootstrap_gate_batch(ctx.h, _dev(ops), _dev(in0), _dev(in1), _dev(out), count,
                                          _stream(stream)), "fhe_bootstrap_gate_batch")


def fhe_bootstrap_gate_plain(ctx, op, in0, in1, out, stream=None):
    _check(lib().fhe_bootstrap_gate_plain(ctx.h, op, _dev(in0), _dev(in1), _dev(out), _stream(stream)),
           "fhe_bootstrap_gate_plain")


def fhe_add(ctx, A, B, R, count, width, stream=None):
    _check(lib().fhe_add(ctx.h, _dev(A), _dev(B), _dev(R), count, width, _stream(stream)), "fhe_add")


def fhe_add_fa(ctx, A, B, R, count, width, stream=None):
    _check(lib().fhe_add_fa(ctx.h, _dev(A), _dev(B), _dev(R), count, width, _stream(stream)), "fhe_add_fa")


def fhe_bootstrap_gate3_batch(ctx, ops, in0, in1, in2, out, count, stream=None):
    _check(lib().fhe_bootstrap_gate3_batch(ctx.h, _dev(ops), _dev(in0), _dev(in1), _dev(in2), _dev(out), count,
                                           _stream(stream)), "fhe_bootstrap_gate3_batch")


def fhe_bootstrap_lut_batch(ctx, tv, inp, out, count, stream=None):
    """Programmable bootstrapping with test vector tv (device uint32[N])."""
    _check(lib().fhe_bootstrap_lut_batch(ctx.h, _dev(tv), _dev(inp), _dev(out), count, _stream(stream)),
           "fhe_bootstrap_lut_batch")


def fhe_bootstrap_gate_batch_noalloc(ctx, ops, in0, in1, out, count, stream=None):
    """fhe_bootstrap_gate_batch with the library's fixed scratch array (allocates nothing; count <= 4096)."""
    _check(lib().fhe_bootstrap_gate_batch_noalloc(ctx.h, _dev(ops), _dev(in0), _dev(in1), _dev(out), count,
                                                  _stream(stream)), "fhe_bootstrap_gate_batch_noalloc")


def fhe_bootstrap_compound_batch(ctx, ops0, ops1, in0, in1, out0, out1, count, stream=None):
    """(out0, out1) = (ops0(in0, in1), ops1(in0, in1)) from one blind rotation per gate pair."""
    _check(lib().fhe_bootstrap_compound_batch(ctx.h, _dev(ops0), _dev(ops1), _dev(in0), _dev(in1), _dev(out0),
                                              _dev(out1), count, _stream(stream)), "fhe_bootstrap_compound_batch")


def fhe_ctx_check(ctx):
    """Raises FheError(FHE_EINVAL) if a kernel met an invalid gate code since the last check."""
    _check(lib().fhe_ctx_check(ctx.h), "fhe_ctx_check")


def fhe_add_compound(ctx, A, B, R, count, width, stream=None):
    """R = (A + B) mod 2^width, ripple carry with compound (XOR, AND) gates."""
    _check(lib().fhe_add_compound(ctx.h, _dev(A), _dev(B), _dev(R), count, width, _stream(stream)),
           "fhe_add_compound")


def fhe_add_numberwise(ctx, A, B, R, count, width, stream=None):
    _check(lib().fhe_add_numberwise(ctx.h, _dev(A), _dev(B), _dev(R), count, width, _stream(stream)),
           "fhe_add_numberwise")


def fhe_mul(ctx, A, B, R, count, width, stream=None):
    _check(lib().fhe_mul(ctx.h, _dev(A), _dev(B), _dev(R), count, width, _stream(stream)), "fhe_mul")


def fhe_mul_tree(ctx, A, B, R, count, width, stream=None):
    _check(lib().fhe_mul_tree(ctx.h, _dev(A), _dev(B), _dev(R), count, width, _stream(stream)), "fhe_mul_tree")


def fhe_mul_karatsuba(ctx, A, B, R, count, width, stream=None):
    """R ([count][2 width][n+1]) = full products A * B by Karatsuba's algorithm."""
    _check(lib().fhe_mul_karatsuba(ctx.h, _dev(A), _dev(B), _dev(R), count, width, _stream(stream)),
           "fhe_mul_karatsuba")


def fhe_matvec(ctx, M, x, y, rows, cols, width, stream=None):
    _check(lib().fhe_matvec(ctx.h, _dev(M), _dev(x), _dev(y), rows, cols, width, _stream(stream)),
           "fhe_matvec")


def fhe_matmul(ctx, A, B, Cm, n, width, stream=None):
    """C = A B mod 2^width (n x n) by Cannon's algorithm."""
    _check(lib().fhe_matmul(ctx.h, _dev(A), _dev(B), _dev(Cm), n, width, _stream(stream)), "fhe_matmul")


def fhe_circuit_schedule(kind, width, count, cu_count=256, rows=0, cols=0):
    """Gates per launch of the level schedule for `count` instances."""
    k = CIRCUIT_KINDS[kind]
    lv = C.c_uint32()
    _check(lib().fhe_circuit_schedule(k, width, rows, cols, count, cu_count, None, 0, C.byref(lv)),
           "fhe_circuit_schedule")
    out = (C.c_uint64 * max(lv.value, 1))()
    _check(lib().fhe_circuit_schedule(k, width, rows, cols, count, cu_count, out, lv.value, C.byref(lv)),
           "fhe_circuit_schedule")
    return [out[i] for i in range(lv.value)]


def fhe_circuit_shape(kind, width, rows=0, cols=0):
    """(gates, levels, widest level) of a circuit; kind in {'add', 'mul', 'matvec', 'mul_tree',
    'karatsuba', 'add_numberwise', 'matmul', 'add_fa'} (matmul: rows = n)."""
    k = CIRCUIT_KINDS[kind]
    g, lv, wd = C.c_uint64(), C.c_uint32(), C.c_uint64()
    _check(lib().fhe_circuit_shape(k, width, rows, cols, C.byref(g), C.byref(lv), C.byref(wd)),
           "fhe_circuit_shape")
    return g.value, lv.value, wd.value


def fhe_ctx_set_timing(ctx, enable):
    _check(lib().fhe_ctx_set_timing(ctx.h, 1 if enable else 0), "fhe_ctx_set_timing")


def fhe_ctx_set_graphs(ctx, enable):
    _check(lib().fhe_ctx_set_graphs(ctx.h, 1 if enable else 0), "fhe_ctx_set_graphs")


# Launch shapes of the blind-rotation kernel (the autotuner's search space):
# (waves_per_gate, gates_per_group, arith), arith 0 = Goldilocks NTT,
# 1 = two-prime NTT.
SHAPES = [(w, g, a) for a in (0, 1) for (w, g) in ((1, 1), (1, 2), (1, 4), (1, 8), (2, 1))] + [(4, 1, 1)]


def fhe_ctx_autotune(ctx, max_width=4096, reps=2):
    _check(lib().fhe_ctx_autotune(ctx.h, max_width, reps), "fhe_ctx_autotune")


def fhe_ctx_launch_config(ctx, width):
    """(waves_per_gate, gates_per_group, arith) used for a batch of `width` gates."""
    c = fhe_launch_config()
    _check(lib().fhe_ctx_launch_config(ctx.h, width, C.byref(c)), "fhe_ctx_launch_config")
    return (c.waves_per_gate, c.gates_per_group, c.arith)


def fhe_ctx_set_launch_config(ctx, min_width, max_width, shape):
    c = fhe_launch_config(*shape)
    _check(lib().fhe_ctx_set_launch_config(ctx.h, min_width, max_width, C.byref(c)),
           "fhe_ctx_set_launch_config")


def fhe_ctx_timing_launches(ctx, max_records=1 << 16):
    """Per-launch records since the last timing call: list of dicts with
    gates, shape (waves_per_gate, gates_per_group), blind_rotate_ms,
    key_switch_ms."""
    buf = (fhe_launch_record * max_records)()
    n = C.c_size_t()
    _check(lib().fhe_ctx_timing_launches(ctx.h, buf, max_records, C.byref(n)), "fhe_ctx_timing_launches")
    return [{"gates": r.gates, "shape": (r.waves_per_gate, r.gates_per_group, r.arith),
             "blind_rotate_ms": r.blind_rotate_ms, "key_switch_ms": r.key_switch_ms}
            for r in buf[:min(n.value, max_records)]]


def fhe_ctx_timing(ctx):
    """(blind_rotate_ms, key_switch_ms, launches, gates) since the last call."""
    br, ks, n, g = C.c_double(), C.c_double(), C.c_uint64(), C.c_uint64()
    _check(lib().fhe_ctx_timing(ctx.h, C.byref(br), C.byref(ks), C.byref(n), C.byref(g)), "fhe_ctx_timing")
    return br.value, ks.value, n.value, g.value


# ---------------------------------------------------------------------------
# Serving
# ---------------------------------------------------------------------------
(FHE_JOB_GATE, FHE_JOB_ADD, FHE_JOB_MUL, FHE_JOB_MATVEC, FHE_JOB_MUL_TREE, FHE_JOB_ADD_FA,
 FHE_JOB_ADD_NUMBERWISE, FHE_JOB_KARATSUBA, FHE_JOB_MATMUL) = range(9)
FHE_JOB_QUEUED, FHE_JOB_RUNNING, FHE_JOB_DONE, FHE_JOB_CANCELLED, FHE_JOB_FAILED = range(5)


class fhe_gate_node(C.Structure):
    _fields_ = [("op", C.c_uint8), ("in0", C.c_uint32), ("in1", C.c_uint32), ("in2", C.c_uint32)]


class Circuit:
    """fhe_circuit: a caller-defined gate DAG run by the level scheduler.
    gates: list of (op, in0, in1) or (op, in0, in1, in2) over wires (inputs
    0..n_inputs-1, gate k writes wire n_inputs + k); outputs: gate wires."""

    def __init__(self, ctx, gates, n_inputs, outputs):
        arr = (fhe_gate_node * len(gates))()
        for k, g in enumerate(gates):
            arr[k] = fhe_gate_node(g[0], g[1], g[2], g[3] if len(g) > 3 else 0xFFFFFFFF)
        outs = (C.c_uint32 * len(outputs))(*outputs)
        h = _vp()
        _check(lib().fhe_circuit_create(ctx.h, C.cast(arr, _vp), len(gates), n_inputs, C.cast(outs, _vp),
                                        len(outputs), C.byref(h)), "fhe_circuit_create")
        self.h, self.ctx, self.n_inputs, self.n_outputs = h.value, ctx, n_inputs, len(outputs)

    def run(self, inp, out, count, stream=None):
        _check(lib().fhe_circuit_run(self.h, _dev(inp), _dev(out), count, _stream(stream)), "fhe_circuit_run")

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.fhe_circuit_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


class fhe_job(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("op", C.c_uint32), ("width", C.c_uint32), ("rows", C.c_uint32),
                ("cols", C.c_uint32), ("in0", _vp), ("in1", _vp), ("out", _vp)]


class Server:
    """fhe_server: continuous batching of jobs on one context."""

    def __init__(self, ctx, hbm_budget_bytes):
        h = _vp()
        _check(lib().fhe_serve_create(ctx.h, hbm_budget_bytes, C.byref(h)), "fhe_serve_create")
        self.h, self.ctx = h.value, ctx

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.fhe_serve_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


def fhe_serve_submit(srv, kind, in0, in1, out, op=0, width=0, rows=0, cols=0):
    j = fhe_job(kind, op, width, rows, cols, _dev(in0), _dev(in1), _dev(out))
    t = C.c_uint64()
    _check(lib().fhe_serve_submit(srv.h, C.byref(j), C.byref(t)), "fhe_serve_submit")
    return t.value


def fhe_serve_poll(srv, ticket):
    """(state, latency_ms); raises for cancelled or failed jobs."""
    st, lat = C.c_int(), C.c_double()
    _check(lib().fhe_serve_poll(srv.h, ticket, C.byref(st), C.byref(lat)), "fhe_serve_poll")
    return st.value, lat.value


def fhe_serve_wait(srv, ticket, timeout_s=600.0):
    _check(lib().fhe_serve_wait(srv.h, ticket, timeout_s), "fhe_serve_wait")


def fhe_serve_job_times(srv, ticket):
    """(queue_ms, service_ms) of a done job."""
    q, v = C.c_double(), C.c_double()
    _check(lib().fhe_serve_job_times(srv.h, ticket, C.byref(q), C.byref(v)), "fhe_serve_job_times")
    return q.value, v.value


def fhe_serve_cancel(srv, ticket):
    _check(lib().fhe_serve_cancel(srv.h, ticket), "fhe_serve_cancel")


def fhe_serve_stats(srv):
    v = [C.c_uint64() for _ in range(5)]
    _check(lib().fhe_serve_stats(srv.h, *[C.byref(x) for x in v]), "fhe_serve_stats")
    return dict(zip(["jobs_done", "gates_done", "launches", "pool_bytes_in_use", "jobs_waiting"], [x.value for x in v]))


def fhe_debug_cmux(bk_i, abar, acc, device=0, arith=0):
    """One CMux step on host arrays with the production kernels of NTT
    arithmetic `arith` (test entry)."""
    b, pb = _host(bk_i, np.uint32)
    a = np.ascontiguousarray(acc, np.uint32).copy()
    _check(lib().fhe_debug_cmux(device, arith, pb, abar, a.ctypes.data), "fhe_debug_cmux")
    return a


VALU_CLASSES = ["v_add_u32", "v_mul_lo_u32", "v_mad_i64_i32", "v_mul_hi_u32", "v_bfe_i32", "v_permlane32_swap"]


def fhe_debug_valu_rate(op, device=0):
    """Issue rate of VALU instruction class op (index into VALU_CLASSES), lane-ops/s."""
    r = C.c_double()
    _check(lib().fhe_debug_valu_rate(device, op, C.byref(r)), "fhe_debug_valu_rate")
    return r.value


def fhe_debug_plan(ctx, kind, width, count=1, rows=0, cols=0):
    """(gates [G][5] uint32 {op, in0, in1, out, in2}, level offsets [L+1]) of
    the plan a circuit entry point runs (test entry)."""
    k = CIRCUIT_KINDS[kind]
    g, lv = C.c_uint64(), C.c_uint32()
    _check(lib().fhe_debug_plan(ctx.h, k, width, rows, cols, count, None, 0, None, 0, C.byref(g), C.byref(lv)),
           "fhe_debug_plan")
    gates = np.zeros((g.value, 5), np.uint32)
    off = np.zeros(lv.value + 1, np.uint32)
    _check(lib().fhe_debug_plan(ctx.h, k, width, rows, cols, count, gates.ctypes.data, g.value, off.ctypes.data,
                                lv.value + 1, C.byref(g), C.byref(lv)), "fhe_debug_plan")
    return gates, off


def fhe_debug_read_wires(ctx, kind, width, A, B, R, wires, count=1, rows=0, cols=0):
    """Samples [n][n+1] on the given wires of a plan after a run on A, B, R (test entry)."""
    w, pw = _host(wires, np.uint32)
    out = np.zeros((w.shape[0], WORDS), np.uint32)
    _check(lib().fhe_debug_read_wires(ctx.h, CIRCUIT_KINDS[kind], width, rows, cols, count, _dev(A), _dev(B),
                                      _dev(R), pw, w.shape[0], out.ctypes.data), "fhe_debug_read_wires")
    return out


# ---------------------------------------------------------------------------
# torch helpers (plumbing: device memory only)
# ---------------------------------------------------------------------------

def to_device(arr, device="cuda:0"):
    """Host uint32/uint8 array -> contiguous device tensor with the same bytes."""
    import torch
    a = np.ascontiguousarray(arr)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a.copy()).to(device)


def to_host(t):
    """Device tensor -> numpy array (uint32 view for int32 tensors)."""
    a = t.detach().cpu().numpy()
    return a.view(np.uint32) if a.dtype == np.int32 else a


def empty_samples(shape, device="cuda:0"):
    import torch
    return torch.empty((*shape, WORDS), dtype=torch.int32, device=device)
