"""FP64 CPU oracle for syndrome-form sum-product decoding (test infrastructure).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package; the decoder product never does.
It shares no code with the HIP decoder.  The arithmetic lives in plain C
(``ldpc_oracle.c``: QC lifting of Sec. III-C and Algorithm 1 of Sec. III-D in
double precision); this module compiles it with gcc and marshals numpy
arrays.  ``octonion.py`` holds the 8-dimensional reconciliation reference
(Sec. II-C.3) in plain numpy.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ldpc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None
_lock = threading.Lock()


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (IEEE double, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.oracle_phi.restype = ctypes.c_double
        lib.oracle_phi.argtypes = [ctypes.c_double]
        lib.oracle_code_build.restype = P
        lib.oracle_code_build.argtypes = [ctypes.c_int, ctypes.c_int, P, ctypes.c_int]
        lib.oracle_code_free.argtypes = [P]
        lib.oracle_code_free.restype = None
        for name in ("oracle_code_n", "oracle_code_m", "oracle_code_edges"):
            getattr(lib, name).restype = ctypes.c_int
            getattr(lib, name).argtypes = [P]
        lib.oracle_code_edge_list.argtypes = [P, P, P]
        lib.oracle_code_edge_list.restype = None
        lib.oracle_syndrome.argtypes = [P, P, P]
        lib.oracle_syndrome.restype = None
        lib.oracle_decode.restype = ctypes.c_int
        lib.oracle_decode.argtypes = [P, P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      P, P, ctypes.POINTER(ctypes.c_int)]
        _lib = lib
        return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def phi(x: float) -> float:
    """Phi(x) = -ln tanh(x/2) on the argument clamped to [1e-7, 30]."""
    return _load().oracle_phi(float(x))


class OracleCode:
    """Explicitly expanded QC parity-check matrix (Sec. III-C lifting)."""

    def __init__(self, base: np.ndarray, Z: int):
        lib = _load()
        self.base = np.ascontiguousarray(base, dtype=np.int32)
        self.mb, self.nb = self.base.shape
        self.Z = int(Z)
        h = lib.oracle_code_build(self.mb, self.nb, _ptr(self.base), self.Z)
        if not h:
            raise ValueError("oracle: invalid base matrix or Z")
        self._h = ctypes.c_void_p(h)
        self.n = lib.oracle_code_n(self._h)
        self.m = lib.oracle_code_m(self._h)
        self.E = lib.oracle_code_edges(self._h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.oracle_code_free(h)
            self._h = None

    def edge_list(self):
        chk = np.empty(self.E, dtype=np.int32)
        var = np.empty(self.E, dtype=np.int32)
        _load().oracle_code_edge_list(self._h, _ptr(chk), _ptr(var))
        return chk, var

    def syndrome(self, x: np.ndarray) -> np.ndarray:
        """H x mod 2 for uint8 words [..., n]."""
        x = np.ascontiguousarray(x, dtype=np.uint8)
        flat = x.reshape(-1, self.n)
        out = np.empty((flat.shape[0], self.m), dtype=np.uint8)
        for f in range(flat.shape[0]):
            _load().oracle_syndrome(self._h, _ptr(flat[f]), _ptr(out[f]))
        return out.reshape(x.shape[:-1] + (self.m,))

    def decode_frame(self, Q, s, max_iters, early_stop=True, check_from=0):
        Qd = np.ascontiguousarray(Q, dtype=np.float64)
        sd = np.ascontiguousarray(s, dtype=np.uint8)
        if Qd.shape != (self.n,) or sd.shape != (self.m,):
            raise ValueError("oracle: frame shapes do not match the code")
        bits = np.empty(self.n, dtype=np.uint8)
        L = np.empty(self.n, dtype=np.float64)
        it = ctypes.c_int(0)
        rc = _load().oracle_decode(self._h, _ptr(Qd), _ptr(sd), int(max_iters),
                                   int(bool(early_stop)), int(check_from),
                                   _ptr(bits), _ptr(L), ctypes.byref(it))
        if rc < 0:
            raise MemoryError("oracle: allocation failed")
        return bits, L, it.value, bool(rc)

    def decode(self, Q, s, max_iters, early_stop=True, check_from=0, threads=1):
        """Decode frames [F][n]; frames may be spread over ``threads`` threads.

        Returns (bits uint8 [F][n], L float64 [F][n], iters int32 [F], converged bool [F]).
        """
        Q = np.asarray(Q)
        s = np.asarray(s)
        F = Q.shape[0]
        bits = np.empty((F, self.n), dtype=np.uint8)
        L = np.empty((F, self.n), dtype=np.float64)
        iters = np.empty(F, dtype=np.int32)
        conv = np.empty(F, dtype=bool)

        def one(f):
            b, l, i, c = self.decode_frame(Q[f], s[f], max_iters, early_stop, check_from)
            bits[f], L[f], iters[f], conv[f] = b, l, i, c

        if threads <= 1 or F == 1:
            for f in range(F):
                one(f)
        else:
            with ThreadPoolExecutor(max_workers=threads) as ex:
                list(ex.map(one, range(F)))
        return bits, L, iters, conv
