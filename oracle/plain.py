"""The plain C oracle (``gls_plain.c``): single-threaded float64 GLS solves of
Eq. (1) with no BLAS, for the tests and the benchmark's CPU baseline.

TEST INFRASTRUCTURE ONLY, like the rest of this package.  ``build()`` compiles
it with gcc into ``oracle/libglsplain.so`` (no fast-math); ``GLSPlain`` has the
interface of ``GLSOracle``: ``GLSPlain(M, XL, Y).solve(XR)`` returns b (m,t,p),
var (m,) and info (m,).
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(HERE, "gls_plain.c")
LIBRARY = os.path.join(HERE, "libglsplain.so")
RANK_TOL = 1e-10

_lib = None


def build(verbose: bool = False) -> str:
    """Compile gls_plain.c (always, like the library's own build)."""
    tmp = LIBRARY + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fno-fast-math", SOURCE, "-o", tmp, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("building the plain C oracle failed:\n" + r.stderr)
    os.replace(tmp, LIBRARY)
    if verbose:
        print(f"built {LIBRARY}", flush=True)
    return LIBRARY


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBRARY) or os.path.getmtime(LIBRARY) < os.path.getmtime(SOURCE):
        build()
    lib = ctypes.CDLL(LIBRARY)
    d, i64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_int
    pd = ctypes.POINTER(ctypes.c_double)
    pi = ctypes.POINTER(ctypes.c_int32)
    lib.gls_plain_work_size.restype = i64
    lib.gls_plain_work_size.argtypes = [i64, i32, i32]
    lib.gls_plain_setup.restype = i64
    lib.gls_plain_setup.argtypes = [i64, i32, i32, pd, i64, pd, i64, pd, i64, pd]
    lib.gls_plain_solve.restype = i32
    lib.gls_plain_solve.argtypes = [pd, i64, i32, i32, i64, pd, i64, pd, pd, pi, d, pd]
    _lib = lib
    return lib


def _ptr(a, kind=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(kind))


class GLSPlain:
    """Eq. (1) by the plain C oracle: Cholesky of M once, then per SNP two
    triangular solves and a pivoted p x p elimination."""

    def __init__(self, M, XL, Y, rank_tol: float = RANK_TOL):
        lib = _load()
        M = np.asfortranarray(np.asarray(M, dtype=np.float64))
        self.n = M.shape[0]
        XL = np.asfortranarray(np.asarray(XL, dtype=np.float64).reshape(self.n, -1))
        Y = np.asarray(Y, dtype=np.float64)
        Y = np.asfortranarray(Y[:, None] if Y.ndim == 1 else Y)
        self.p = XL.shape[1] + 1
        self.t = Y.shape[1]
        self.rank_tol = rank_tol
        self.work = np.empty(lib.gls_plain_work_size(self.n, self.p, self.t))
        rc = lib.gls_plain_setup(self.n, self.p, self.t, _ptr(M), self.n, _ptr(XL), self.n, _ptr(Y), self.n,
                                 _ptr(self.work))
        if rc != 0:
            raise np.linalg.LinAlgError(f"M is not positive definite (pivot {rc})" if rc > 0 else "bad sizes")

    def solve(self, XR):
        """b (m,t,p), var (m,), info (m,) int32 for SNP-major dosages XR (m,n)."""
        lib = _load()
        XR = np.ascontiguousarray(np.asarray(XR, dtype=np.float64))
        m = XR.shape[0]
        b = np.empty((m, self.t, self.p))
        var = np.empty(m)
        info = np.empty(m, dtype=np.int32)
        tmp = np.empty(self.n)
        rc = lib.gls_plain_solve(_ptr(self.work), self.n, self.p, self.t, m, _ptr(XR), self.n, _ptr(b), _ptr(var),
                                 _ptr(info, ctypes.c_int32), self.rank_tol, _ptr(tmp))
        if rc != 0:
            raise ValueError("bad sizes")
        return b, var, info
