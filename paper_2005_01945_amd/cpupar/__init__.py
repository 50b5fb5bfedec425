"""The paper's CPU parallel framework (Sec. IV) as a host baseline: one gate
bootstrap per core (exact two-prime NTT products, the same words as the GPU
path), independent gates, numbers and partial products spread over the cores
with OpenMP.  Used by the benchmark beside the GPU figures; the GPU library
never calls it."""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfhe_cpupar.so")
WORDS = 501
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built (python -m paper_2005_01945_amd.cpupar.build)")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.cpupar_create.restype = C.c_int
        L.cpupar_create.argtypes = [vp, vp, C.POINTER(vp)]
        L.cpupar_destroy.restype = None
        L.cpupar_destroy.argtypes = [vp]
        L.cpupar_bootstrap_gates.restype = C.c_int
        L.cpupar_bootstrap_gates.argtypes = [vp, vp, vp, vp, vp, C.c_size_t, C.c_int]
        for name in ("cpupar_add", "cpupar_mul"):
            f = getattr(L, name)
            f.restype = C.c_int
            f.argtypes = [vp, vp, vp, vp, C.c_size_t, C.c_uint32, C.c_int]
        _lib = L
    return _lib


def _u32(a):
    return np.ascontiguousarray(a, dtype=np.uint32)


class CpuParallel:
    """Keys prepared for the host baseline: bk [n][4][2][N], ksk [N][8][4][n+1]
    (the layouts fhe_cloud_key_export writes)."""

    def __init__(self, bk, ksk):
        b, k = _u32(bk), _u32(ksk)
        h = C.c_void_p()
        if lib().cpupar_create(b.ctypes.data, k.ctypes.data, C.byref(h)):
            raise RuntimeError("cpupar_create failed")
        self.h = h.value

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.cpupar_destroy(self.h)
            self.h = None

    def bootstrap(self, ops, in0, in1, threads=0):
        o = np.ascontiguousarray(ops, dtype=np.uint8)
        a = _u32(in0).reshape(-1, WORDS)
        b = _u32(in1).reshape(-1, WORDS)
        out = np.empty((o.size, WORDS), np.uint32)
        if lib().cpupar_bootstrap_gates(self.h, o.ctypes.data, a.ctypes.data, b.ctypes.data, out.ctypes.data,
                                        o.size, threads):
            raise ValueError("cpupar_bootstrap_gates: bad arguments")
        return out

    def _binary(self, fn, A, B, width, threads):
        a = _u32(A).reshape(-1, width, WORDS)
        b = _u32(B).reshape(-1, width, WORDS)
        out = np.empty_like(a)
        if fn(self.h, a.ctypes.data, b.ctypes.data, out.ctypes.data, a.shape[0], width, threads):
            raise ValueError("bad arguments")
        return out

    def add(self, A, B, width, threads=0):
        """(A + B) mod 2^width: numbers across threads, bits in carry order (Sec. IV-A)."""
        return self._binary(lib().cpupar_add, A, B, width, threads)

    def mul(self, A, B, width, threads=0):
        """(A * B) mod 2^width: partial-product ANDs across threads, accumulation in order (Sec. IV-B)."""
        return self._binary(lib().cpupar_mul, A, B, width, threads)
