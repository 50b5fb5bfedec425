"""CPU oracle for TFHE gate bootstrapping — TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct C (schoolbook negacyclic products in wrapping
uint32 arithmetic) behind a ctypes wrapper.  Only the tests, the smoke check
and the benchmark's CPU-baseline leg may import this package; the product
library never does, and the two share no code.

Each wrapper cites what its C function follows; see tfhe_oracle.h.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

AND, NAND, OR, NOR, XOR, XNOR, ANDNY, ANDYN, ORNY, ORYN = range(10)
GATE_NAMES = ["AND", "NAND", "OR", "NOR", "XOR", "XNOR", "ANDNY", "ANDYN", "ORNY", "ORYN"]
MAJ, XOR3 = 10, 11  # three-input gates: majority and parity
MU = 1 << 29


class Params(C.Structure):
    _fields_ = [("n", C.c_int32), ("N", C.c_int32), ("bk_l", C.c_int32),
                ("bk_bgbit", C.c_int32), ("ks_t", C.c_int32), ("ks_basebit", C.c_int32),
                ("lwe_stdev", C.c_double), ("bk_stdev", C.c_double)]


class _Keys(C.Structure):
    _fields_ = [("P", Params), ("seed", C.c_uint64),
                ("lwe_key", C.POINTER(C.c_int32)), ("tlwe_key", C.POINTER(C.c_int32)),
                ("bk", C.POINTER(C.c_uint32)), ("ksk", C.POINTER(C.c_uint32))]


def _u32p(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint32))


def _i32p(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _u8p(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint8))


def lib():
    global _lib
    if _lib is None:
        path = os.path.join(_HERE, "libtfhe_oracle.so")
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        KP = C.POINTER(_Keys)
        PP = C.POINTER(Params)
        u32p, i32p, u8p = C.POINTER(C.c_uint32), C.POINTER(C.c_int32), C.POINTER(C.c_uint8)
        sig = {
            "or_mix64": (C.c_uint64, [C.c_uint64]),
            "or_draw": (C.c_uint64, [C.c_uint64, C.c_uint64, C.c_uint64]),
            "or_gaussian": (C.c_double, [C.c_uint64, C.c_uint64, C.c_uint64]),
            "or_torus_from_double": (C.c_uint32, [C.c_double]),
            "or_default_params": (None, [PP]),
            "or_keygen": (C.c_int, [PP, C.c_uint64, i32p, i32p, KP]),
            "or_keys_free": (None, [KP]),
            "or_encrypt_bits": (None, [KP, u8p, C.c_size_t, C.c_uint64, u32p]),
            "or_phase": (None, [KP, u32p, C.c_size_t, i32p]),
            "or_decrypt_bits": (None, [KP, u32p, C.c_size_t, u8p]),
            "or_negacyclic_mul": (None, [C.c_int32, u32p, u32p, u32p]),
            "or_rotate": (None, [C.c_int32, u32p, C.c_int32, u32p]),
            "or_gadget_decompose": (None, [PP, C.c_uint32, i32p]),
            "or_modswitch": (C.c_uint32, [PP, C.c_uint32]),
            "or_gate_combine": (None, [PP, C.c_int, u32p, u32p, u32p]),
            "or_external_product_cmux": (None, [PP, u32p, C.c_int32, u32p]),
            "or_blind_rotate": (None, [KP, u32p, u32p]),
            "or_blind_rotate_tv": (None, [KP, u32p, u32p, u32p]),
            "or_sample_extract": (None, [PP, u32p, u32p]),
            "or_sample_extract_at": (None, [PP, u32p, C.c_int32, u32p]),
            "or_compound_combine": (C.c_int, [PP, C.c_int, u32p, u32p]),
            "or_bootstrap_compounds": (C.c_int, [KP, u8p, u32p, u32p, u32p, C.c_size_t, C.c_int]),
            "or_key_switch": (None, [KP, u32p, u32p]),
            "or_bootstrap_gate": (None, [KP, C.c_int, u32p, u32p, u32p]),
            "or_bootstrap_gates": (None, [KP, u8p, u32p, u32p, u32p, C.c_size_t, C.c_int]),
            "or_circuit_add": (None, [KP, u32p, u32p, u32p, C.c_size_t, C.c_int32, C.c_int]),
            "or_circuit_mul": (None, [KP, u32p, u32p, u32p, C.c_size_t, C.c_int32, C.c_int]),
            "or_circuit_mul_tree": (None, [KP, u32p, u32p, u32p, C.c_size_t, C.c_int32, C.c_int]),
            "or_circuit_karatsuba": (None, [KP, u32p, u32p, u32p, C.c_size_t, C.c_int32, C.c_int]),
            "or_circuit_add_numberwise": (None, [KP, u32p, u32p, u32p, C.c_size_t, C.c_int32, C.c_int]),
            "or_circuit_matmul": (None, [KP, u32p, u32p, u32p, C.c_int32, C.c_int32, C.c_int]),
            "or_circuit_add_fa": (None, [KP, u32p, u32p, u32p, C.c_size_t, C.c_int32, C.c_int]),
            "or_circuit_add_compound": (None, [KP, u32p, u32p, u32p, C.c_size_t, C.c_int32, C.c_int]),
            "or_bootstrap_lut": (None, [KP, u32p, u32p, u32p, C.c_size_t, C.c_int]),
            "or_bootstrap_gates3": (None, [KP, u8p, u32p, u32p, u32p, u32p, C.c_size_t, C.c_int]),
            "or_circuit_eval_plain": (C.c_long, [C.c_int, C.c_int32, C.c_int32, C.c_int32, u8p, u8p]),
            "or_circuit_matvec": (None, [KP, u32p, u32p, u32p, C.c_int32, C.c_int32, C.c_int32, C.c_int]),
            "or_circuit_gate_count": (C.c_long, [C.c_int, C.c_int32, C.c_int32, C.c_int32]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def default_params(**overrides) -> Params:
    """TFHE's 110-bit gate-bootstrapping parameters (paper Sec. VII)."""
    P = Params()
    lib().or_default_params(C.byref(P))
    for k, v in overrides.items():
        setattr(P, k, v)
    return P


def mix64(z: int) -> int:
    return lib().or_mix64(z)


def draw(seed: int, stream: int, idx: int) -> int:
    return lib().or_draw(seed, stream, idx)


def gaussian(seed: int, stream: int, idx: int) -> float:
    return lib().or_gaussian(seed, stream, idx)


def torus_from_double(x: float) -> int:
    return lib().or_torus_from_double(x)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


class Keys:
    """Secret and cloud keys (paper Sec. II-A; TFHE's TGSW bootstrapping key
    and LWE key-switching key)."""

    def __init__(self, seed: int = 0, params: Params = None, lwe_key=None, tlwe_key=None):
        self.P = params if params is not None else default_params()
        self._k = _Keys()
        lk = None if lwe_key is None else _c(lwe_key, np.int32)
        tk = None if tlwe_key is None else _c(tlwe_key, np.int32)
        rc = lib().or_keygen(C.byref(self.P), seed,
                             _i32p(lk) if lk is not None else None,
                             _i32p(tk) if tk is not None else None, C.byref(self._k))
        if rc != 0:
            raise MemoryError("oracle keygen failed")
        self.seed = seed
        n, N, L2 = self.P.n, self.P.N, 2 * self.P.bk_l
        B = 1 << self.P.ks_basebit
        self.lwe_key = np.ctypeslib.as_array(self._k.lwe_key, shape=(n,))
        self.tlwe_key = np.ctypeslib.as_array(self._k.tlwe_key, shape=(N,))
        self.bk = np.ctypeslib.as_array(self._k.bk, shape=(n, L2, 2, N))
        self.ksk = np.ctypeslib.as_array(self._k.ksk, shape=(N, self.P.ks_t, B, n + 1))

    @property
    def width(self) -> int:
        return self.P.n + 1

    def __del__(self):
        try:
            if self._k.bk:
                lib().or_keys_free(C.byref(self._k))
        except Exception:
            pass

    def ref(self):
        return C.byref(self._k)

    # --- encryption (Sec. II-A) ---
    def encrypt_bits(self, bits, nonce: int = 0) -> np.ndarray:
        b = _c(bits, np.uint8).reshape(-1)
        out = np.empty((b.size, self.width), np.uint32)
        lib().or_encrypt_bits(self.ref(), _u8p(b), b.size, nonce, _u32p(out))
        return out

    def encrypt_uint(self, values, width: int, nonce: int = 0) -> np.ndarray:
        """An integer as `width` samples, LSB first (Sec. II-A: an n-bit integer
        becomes n LWE samples)."""
        v = np.asarray(values, dtype=np.uint64).reshape(-1)
        bits = ((v[:, None] >> np.arange(width, dtype=np.uint64)[None, :]) & np.uint64(1)).astype(np.uint8)
        return self.encrypt_bits(bits.reshape(-1), nonce).reshape(v.size, width, self.width)

    def phase(self, ct) -> np.ndarray:
        c = _c(ct, np.uint32).reshape(-1, self.width)
        out = np.empty(c.shape[0], np.int32)
        lib().or_phase(self.ref(), _u32p(c), c.shape[0], _i32p(out))
        return out

    def decrypt_bits(self, ct) -> np.ndarray:
        c = _c(ct, np.uint32).reshape(-1, self.width)
        out = np.empty(c.shape[0], np.uint8)
        lib().or_decrypt_bits(self.ref(), _u32p(c), c.shape[0], _u8p(out))
        return out

    def decrypt_uint(self, ct, width: int) -> np.ndarray:
        bits = self.decrypt_bits(ct).reshape(-1, width).astype(np.uint64)
        return (bits << np.arange(width, dtype=np.uint64)[None, :]).sum(axis=1, dtype=np.uint64)

    # --- bootstrapping pieces ---
    def blind_rotate(self, lwe_in, tv=None) -> np.ndarray:
        """Blind rotation of the gate test vector (mu everywhere) or of tv[N]."""
        x = _c(lwe_in, np.uint32)
        acc = np.empty(2 * self.P.N, np.uint32)
        if tv is None:
            lib().or_blind_rotate(self.ref(), _u32p(x), _u32p(acc))
        else:
            v = _c(tv, np.uint32)
            assert v.size == self.P.N
            lib().or_blind_rotate_tv(self.ref(), _u32p(x), _u32p(v), _u32p(acc))
        return acc.reshape(2, self.P.N)

    def sample_extract(self, acc) -> np.ndarray:
        a = _c(acc, np.uint32).reshape(-1)
        out = np.empty(self.P.N + 1, np.uint32)
        lib().or_sample_extract(C.byref(self.P), _u32p(a), _u32p(out))
        return out

    def sample_extract_at(self, acc, m: int) -> np.ndarray:
        """LWE sample (under the TLWE key's coefficients) of coefficient m of the TLWE sample acc."""
        a = _c(acc, np.uint32).reshape(-1)
        out = np.empty(self.P.N + 1, np.uint32)
        lib().or_sample_extract_at(C.byref(self.P), _u32p(a), m, _u32p(out))
        return out

    def key_switch(self, lwe_big) -> np.ndarray:
        a = _c(lwe_big, np.uint32)
        out = np.empty(self.width, np.uint32)
        lib().or_key_switch(self.ref(), _u32p(a), _u32p(out))
        return out

    def bootstrap(self, ops, in0, in1, threads: int = 0) -> np.ndarray:
        """Gate bootstrapping of each (op, in0, in1): linear combination,
        blind rotation, sample extraction, key switching."""
        o = _c(ops, np.uint8).reshape(-1)
        a = _c(in0, np.uint32).reshape(-1, self.width)
        b = _c(in1, np.uint32).reshape(-1, self.width)
        assert a.shape[0] == o.size and b.shape[0] == o.size
        out = np.empty((o.size, self.width), np.uint32)
        lib().or_bootstrap_gates(self.ref(), _u8p(o), _u32p(a), _u32p(b), _u32p(out), o.size, threads)
        return out

    def bootstrap_compound(self, ops, in0, in1, threads: int = 0) -> np.ndarray:
        """Compound gates (Sec. V-A-3): ops [count][2] symmetric codes; out
        [count][2][n+1] = (ops[g][0](in0[g], in1[g]), ops[g][1](in0[g], in1[g]))
        from one blind rotation per g."""
        o = _c(ops, np.uint8).reshape(-1, 2)
        a = _c(in0, np.uint32).reshape(-1, self.width)
        b = _c(in1, np.uint32).reshape(-1, self.width)
        assert a.shape[0] == o.shape[0] and b.shape[0] == o.shape[0]
        out = np.empty((o.shape[0], 2, self.width), np.uint32)
        rc = lib().or_bootstrap_compounds(self.ref(), _u8p(o), _u32p(a), _u32p(b), _u32p(out), o.shape[0], threads)
        if rc:
            raise ValueError("compound gates take symmetric codes only (AND, NAND, OR, NOR, XOR, XNOR)")
        return out

    # --- circuits ---
    def add(self, A, B, width: int, threads: int = 0) -> np.ndarray:
        a = _c(A, np.uint32).reshape(-1, width, self.width)
        b = _c(B, np.uint32).reshape(-1, width, self.width)
        out = np.empty_like(a)
        lib().or_circuit_add(self.ref(), _u32p(a), _u32p(b), _u32p(out), a.shape[0], width, threads)
        return out

    def mul(self, A, B, width: int, threads: int = 0) -> np.ndarray:
        a = _c(A, np.uint32).reshape(-1, width, self.width)
        b = _c(B, np.uint32).reshape(-1, width, self.width)
        out = np.empty_like(a)
        lib().or_circuit_mul(self.ref(), _u32p(a), _u32p(b), _u32p(out), a.shape[0], width, threads)
        return out

    def mul_tree(self, A, B, width: int, threads: int = 0) -> np.ndarray:
        """Low width bits of A*B, partial products summed by a tree (Sec. V-B-2)."""
        a = _c(A, np.uint32).reshape(-1, width, self.width)
        b = _c(B, np.uint32).reshape(-1, width, self.width)
        out = np.empty_like(a)
        lib().or_circuit_mul_tree(self.ref(), _u32p(a), _u32p(b), _u32p(out), a.shape[0], width, threads)
        return out

    def bootstrap_lut(self, tv, ct, threads: int = 0) -> np.ndarray:
        """Programmable bootstrapping of samples ct [count][n+1] with test vector tv[N]."""
        v = _c(tv, np.uint32)
        c = _c(ct, np.uint32).reshape(-1, self.width)
        out = np.empty_like(c)
        lib().or_bootstrap_lut(self.ref(), _u32p(v), _u32p(c), _u32p(out), c.shape[0], threads)
        return out

    def add_fa(self, A, B, width: int, threads: int = 0) -> np.ndarray:
        """(A + B) mod 2^width, ripple carry of full-adder gates (MAJ, XOR3)."""
        a = _c(A, np.uint32).reshape(-1, width, self.width)
        b = _c(B, np.uint32).reshape(-1, width, self.width)
        out = np.empty_like(a)
        lib().or_circuit_add_fa(self.ref(), _u32p(a), _u32p(b), _u32p(out), a.shape[0], width, threads)
        return out

    def add_compound(self, A, B, width: int, threads: int = 0) -> np.ndarray:
        """(A + B) mod 2^width, eqs. (1)-(2) with compound (XOR, AND) gates (Sec. V-A-3)."""
        a = _c(A, np.uint32).reshape(-1, width, self.width)
        b = _c(B, np.uint32).reshape(-1, width, self.width)
        out = np.empty_like(a)
        lib().or_circuit_add_compound(self.ref(), _u32p(a), _u32p(b), _u32p(out), a.shape[0], width, threads)
        return out

    def bootstrap3(self, ops, in0, in1, in2, threads: int = 0) -> np.ndarray:
        """Bootstrapped gates of up to three inputs (MAJ = 10, XOR3 = 11)."""
        o = _c(ops, np.uint8)
        a = _c(in0, np.uint32).reshape(-1, self.width)
        b = _c(in1, np.uint32).reshape(-1, self.width)
        c = _c(in2, np.uint32).reshape(-1, self.width)
        out = np.empty((o.size, self.width), np.uint32)
        lib().or_bootstrap_gates3(self.ref(), _u8p(o), _u32p(a), _u32p(b), _u32p(c), _u32p(out), o.size, threads)
        return out

    def add_numberwise(self, A, B, width: int, threads: int = 0) -> np.ndarray:
        """(A + B) mod 2^width by number-wise addition (GPU_n, Sec. V-B-1)."""
        a = _c(A, np.uint32).reshape(-1, width, self.width)
        b = _c(B, np.uint32).reshape(-1, width, self.width)
        out = np.empty_like(a)
        lib().or_circuit_add_numberwise(self.ref(), _u32p(a), _u32p(b), _u32p(out), a.shape[0], width, threads)
        return out

    def karatsuba(self, A, B, width: int, threads: int = 0) -> np.ndarray:
        """Full 2 width-bit product by Karatsuba's algorithm (Sec. III-B-2)."""
        a = _c(A, np.uint32).reshape(-1, width, self.width)
        b = _c(B, np.uint32).reshape(-1, width, self.width)
        out = np.empty((a.shape[0], 2 * width, self.width), np.uint32)
        lib().or_circuit_karatsuba(self.ref(), _u32p(a), _u32p(b), _u32p(out), a.shape[0], width, threads)
        return out

    def matmul(self, A, B, n: int, width: int, threads: int = 0) -> np.ndarray:
        """C = A B mod 2^width, n x n matrices, by Cannon's algorithm (Sec. V-B-3)."""
        a = _c(A, np.uint32).reshape(n, n, width, self.width)
        b = _c(B, np.uint32).reshape(n, n, width, self.width)
        out = np.empty_like(a)
        lib().or_circuit_matmul(self.ref(), _u32p(a), _u32p(b), _u32p(out), n, width, threads)
        return out

    def matvec(self, M, x, rows: int, cols: int, width: int, threads: int = 0) -> np.ndarray:
        m = _c(M, np.uint32).reshape(rows, cols, width, self.width)
        v = _c(x, np.uint32).reshape(cols, width, self.width)
        out = np.empty((rows, width, self.width), np.uint32)
        lib().or_circuit_matvec(self.ref(), _u32p(m), _u32p(v), _u32p(out), rows, cols, width, threads)
        return out


# --- free functions over the ring and the gate pieces ---
def negacyclic_mul(P, Q) -> np.ndarray:
    p = _c(P, np.uint32)
    q = _c(Q, np.uint32)
    assert p.size == q.size
    out = np.empty_like(p)
    lib().or_negacyclic_mul(p.size, _u32p(p), _u32p(q), _u32p(out))
    return out


def compound_combine(op: int, acc, params: Params = None) -> np.ndarray:
    """The compound gate's N-dimensional sample of symmetric code op from the
    rotated accumulator acc [2][N] (before key switching)."""
    P = params if params is not None else default_params()
    a = _c(acc, np.uint32).reshape(-1)
    out = np.empty(P.N + 1, np.uint32)
    if lib().or_compound_combine(C.byref(P), op, _u32p(a), _u32p(out)):
        raise ValueError("not a symmetric gate code")
    return out


def rotate(P, a: int) -> np.ndarray:
    p = _c(P, np.uint32)
    out = np.empty_like(p)
    lib().or_rotate(p.size, _u32p(p), a, _u32p(out))
    return out


def gadget_decompose(x: int, params: Params = None):
    P = params if params is not None else default_params()
    d = np.empty(P.bk_l, np.int32)
    lib().or_gadget_decompose(C.byref(P), x, _i32p(d))
    return d


def modswitch(x: int, params: Params = None) -> int:
    P = params if params is not None else default_params()
    return lib().or_modswitch(C.byref(P), x)


def gate_combine(op: int, c1, c2, params: Params = None) -> np.ndarray:
    P = params if params is not None else default_params()
    a = _c(c1, np.uint32)
    b = _c(c2, np.uint32)
    out = np.empty_like(a)
    lib().or_gate_combine(C.byref(P), op, _u32p(a), _u32p(b), _u32p(out))
    return out


def cmux(bk_i, abar: int, acc, params: Params = None) -> np.ndarray:
    """One CMux step acc += BK_i [x] (X^abar acc - acc); bk_i is [2l][2][N]."""
    P = params if params is not None else default_params()
    bk = _c(bk_i, np.uint32)
    a = _c(acc, np.uint32).copy()
    lib().or_external_product_cmux(C.byref(P), _u32p(bk), abar, _u32p(a))
    return a


def circuit_gate_count(kind: str, width: int, rows: int = 0, cols: int = 0) -> int:
    k = {"add": 0, "mul": 1, "matvec": 2, "mul_tree": 3, "karatsuba": 4, "add_numberwise": 5,
         "matmul": 6, "add_fa": 7, "add_compound": 8}[kind]
    return lib().or_circuit_gate_count(k, width, rows, cols)


def circuit_eval_plain(kind: str, width: int, operand_bits, rows: int = 0, cols: int = 0) -> np.ndarray:
    """A circuit's gates evaluated on plaintext bits (uint8 0/1, operands LSB
    first, A then B or M then x; matmul: rows = n); returns the result bits."""
    k = {"add": 0, "mul": 1, "matvec": 2, "mul_tree": 3, "karatsuba": 4, "add_numberwise": 5,
         "matmul": 6, "add_fa": 7, "add_compound": 8}[kind]
    bits = _c(operand_bits, np.uint8)
    nout = {"matvec": rows * width, "matmul": rows * rows * width, "karatsuba": 2 * width}.get(kind, width)
    out = np.empty(nout, np.uint8)
    got = lib().or_circuit_eval_plain(k, width, rows, cols, _u8p(bits), _u8p(out))
    assert got == nout
    return out
