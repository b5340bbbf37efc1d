"""CPU FP64 oracle for the delayed-update Cholesky / LU library.

TEST INFRASTRUCTURE ONLY.  The product path never imports this package: only
the tests, the package's ``smoke()`` check and the benchmark's CPU-baseline leg
do.  The numerical work is the plain C in ``oracle.c`` (textbook algorithms in
IEEE binary64); this module only builds it with gcc and marshals numpy arrays.
It shares no code with the GPU library.

Paper: C. Camarero, arXiv 1812.02056.  Each wrapper names the passage its C
routine follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_CFLAGS = ["-O2", "-fPIC", "-shared", "-std=c11", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-Wall"]


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *_CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        i64, dp, vp = ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p
        lib.oracle_chol.argtypes = [i64, vp, i64, vp, i64]
        lib.oracle_chol.restype = ctypes.c_int
        lib.oracle_lu.argtypes = [i64, vp, i64, vp, i64]
        lib.oracle_lu.restype = ctypes.c_int
        lib.oracle_chol_solve.argtypes = [i64, i64, vp, i64, vp, i64, vp, i64]
        lib.oracle_chol_solve.restype = None
        lib.oracle_lu_solve.argtypes = [i64, i64, vp, i64, vp, i64, vp, i64]
        lib.oracle_lu_solve.restype = None
        lib.oracle_chol_alg1.argtypes = [i64, i64, vp, i64, vp, i64]
        lib.oracle_chol_alg1.restype = i64
        lib.oracle_lu_alg2.argtypes = [i64, i64, vp, i64, vp, i64, vp, i64]
        lib.oracle_lu_alg2.restype = i64
        lib.oracle_syrk_update.argtypes = [i64, i64, vp, i64, vp, i64]
        lib.oracle_syrk_update.restype = None
        lib.oracle_gemm_update.argtypes = [i64, i64, vp, i64, vp, i64, vp, i64]
        lib.oracle_gemm_update.restype = None
        lib.oracle_qr_alg3.argtypes = [i64, i64, i64, vp, i64, vp, i64, vp, i64, ctypes.POINTER(ctypes.c_int)]
        lib.oracle_qr_alg3.restype = i64
        lib.oracle_qr_project.argtypes = [i64, i64, i64, vp, i64, vp, i64, vp, i64]
        lib.oracle_qr_project.restype = None
        lib.oracle_round_f32.argtypes = [ctypes.c_double]
        lib.oracle_round_f32.restype = ctypes.c_double
        lib.oracle_round_bf16.argtypes = [ctypes.c_double]
        lib.oracle_round_bf16.restype = ctypes.c_double
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = ctypes.c_int
        _ = dp
        _lib = lib
    return _lib


def _colmajor(a) -> np.ndarray:
    """A Fortran-ordered float64 copy (column-major, leading dimension = rows)."""
    return np.array(a, dtype=np.float64, order="F", copy=True)


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def chol(A):
    """Cholesky factor L (lower, zero strict upper) and LAPACK-style info.

    Plain definition A = L L^T (Introduction), computed as the paper's
    Cholesky-Crout special case of Algorithm 1 (s = n, Sec. 2)."""
    A = _colmajor(A)
    n = A.shape[0]
    L = np.zeros((n, n), dtype=np.float64, order="F")
    info = _load().oracle_chol(n, _p(A), max(n, 1), _p(L), max(n, 1))
    return L, int(info)


def lu(A):
    """Doolittle LU without pivoting, packed (strict lower = unit-L, upper = U)."""
    A = _colmajor(A)
    n = A.shape[0]
    LU = np.zeros((n, n), dtype=np.float64, order="F")
    info = _load().oracle_lu(n, _p(A), max(n, 1), _p(LU), max(n, 1))
    return LU, int(info)


def chol_solve(L, B):
    """X with L L^T X = B (forward then backward substitution)."""
    L = _colmajor(L)
    B = _colmajor(np.asarray(B).reshape(L.shape[0], -1))
    n, nrhs = B.shape
    X = np.zeros((n, nrhs), dtype=np.float64, order="F")
    _load().oracle_chol_solve(n, nrhs, _p(L), max(n, 1), _p(B), max(n, 1), _p(X), max(n, 1))
    return X


def lu_solve(LU, B):
    """X with L U X = B for Doolittle-packed LU."""
    LU = _colmajor(LU)
    B = _colmajor(np.asarray(B).reshape(LU.shape[0], -1))
    n, nrhs = B.shape
    X = np.zeros((n, nrhs), dtype=np.float64, order="F")
    _load().oracle_lu_solve(n, nrhs, _p(LU), max(n, 1), _p(B), max(n, 1), _p(X), max(n, 1))
    return X


def chol_alg1(A, s: int):
    """Algorithm 1 (Sec. 2) with step s; returns (L, number of deferred updates)."""
    A = _colmajor(A)
    n = A.shape[0]
    L = np.zeros((n, n), dtype=np.float64, order="F")
    nup = _load().oracle_chol_alg1(n, int(s), _p(A), max(n, 1), _p(L), max(n, 1))
    return L, int(nup)


def lu_alg2(A, s: int):
    """Algorithm 2 (Sec. 2) with step s; returns Crout (L, U, updates)."""
    A = _colmajor(A)
    n = A.shape[0]
    L = np.zeros((n, n), dtype=np.float64, order="F")
    U = np.zeros((n, n), dtype=np.float64, order="F")
    nup = _load().oracle_lu_alg2(n, int(s), _p(A), max(n, 1), _p(L), max(n, 1), _p(U), max(n, 1))
    return L, U, int(nup)


def syrk_update(C, P):
    """tril(C) - tril(P P^T): one deferred update of Algorithm 1 (Sec. 2)."""
    C = _colmajor(C)
    P = _colmajor(P)
    m, w = P.shape
    _load().oracle_syrk_update(m, w, _p(C), max(m, 1), _p(P), max(m, 1))
    return C


def gemm_update(C, X, Y):
    """C - X Y: one deferred update of Algorithm 2 (Sec. 2)."""
    C = _colmajor(C)
    X = _colmajor(X)
    Y = _colmajor(Y)
    m, w = X.shape
    _load().oracle_gemm_update(m, w, _p(C), max(m, 1), _p(X), max(m, 1), _p(Y), max(w, 1))
    return C


def qr_alg3(A, s: int):
    """Algorithm 3 (Sec. 2) with step s on an m x n matrix (m >= n).
    Returns (Q, R, block_projections, info); R = Q^T A in full."""
    A = _colmajor(A)
    m, n = A.shape
    if m < n:
        raise ValueError("qr_alg3 needs m >= n")
    Q = np.zeros((m, n), order="F")
    R = np.zeros((n, n), order="F")
    info = ctypes.c_int(0)
    k = _load().oracle_qr_alg3(m, n, int(s), _p(A), max(1, m), _p(Q), max(1, m), _p(R), max(1, n),
                               ctypes.byref(info))
    if k < 0:
        raise MemoryError("oracle_qr_alg3")
    return Q, R, int(k), int(info.value)


def qr_project(Bq, Bm):
    """One block projection of Algorithm 3 (Sec. 2): C = Bq^T Bm, Bm - Bq C.
    Returns (Bm_new, C)."""
    Bq = _colmajor(Bq)
    Bm = _colmajor(Bm)
    m, w = Bq.shape
    k = Bm.shape[1]
    C = np.zeros((w, k), order="F")
    _load().oracle_qr_project(m, w, k, _p(Bq), max(1, m), _p(Bm), max(1, m), _p(C), max(1, w))
    return Bm, C


def round_f32(x):
    f = _load().oracle_round_f32
    return np.vectorize(lambda v: f(float(v)), otypes=[np.float64])(np.asarray(x, dtype=np.float64))


def round_bf16(x):
    f = _load().oracle_round_bf16
    return np.vectorize(lambda v: f(float(v)), otypes=[np.float64])(np.asarray(x, dtype=np.float64))


# ---------------------------------------------------------------------------
# Error measures used to state every result (plain numpy, FP64).
# ---------------------------------------------------------------------------

def rel_lower(L, Lref) -> float:
    """||tril(L - Lref)||_F / ||tril(Lref)||_F."""
    d = np.tril(np.asarray(L, np.float64) - np.asarray(Lref, np.float64))
    den = np.linalg.norm(np.tril(np.asarray(Lref, np.float64)))
    return float(np.linalg.norm(d) / den) if den > 0 else float(np.linalg.norm(d))


def bwd_chol(A, L) -> float:
    """||A - L L^T||_F / ||A||_F over the full symmetric A."""
    L = np.tril(np.asarray(L, np.float64))
    A = np.asarray(A, np.float64)
    return float(np.linalg.norm(A - L @ L.T) / np.linalg.norm(A))


def bwd_lu(A, LU) -> float:
    """||A - L U||_F / ||A||_F for Doolittle-packed LU."""
    LU = np.asarray(LU, np.float64)
    L = np.tril(LU, -1) + np.eye(LU.shape[0])
    U = np.triu(LU)
    A = np.asarray(A, np.float64)
    return float(np.linalg.norm(A - L @ U) / np.linalg.norm(A))


def fwd_x(X, Xref) -> float:
    """||X - Xref||_inf / ||Xref||_inf (max-norm over all entries)."""
    X = np.asarray(X, np.float64)
    Xref = np.asarray(Xref, np.float64)
    return float(np.max(np.abs(X - Xref)) / np.max(np.abs(Xref)))


def bwd_x(A, X, B) -> float:
    """max over columns of ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf)."""
    A = np.asarray(A, np.float64)
    X = np.asarray(X, np.float64).reshape(A.shape[0], -1)
    B = np.asarray(B, np.float64).reshape(A.shape[0], -1)
    R = B - A @ X
    an = np.max(np.sum(np.abs(A), axis=1))
    out = 0.0
    for j in range(X.shape[1]):
        den = an * np.max(np.abs(X[:, j])) + np.max(np.abs(B[:, j]))
        out = max(out, float(np.max(np.abs(R[:, j])) / den) if den > 0 else 0.0)
    return out
