"""Thin Python binding of libfastfact (include/fastfact.h) over ctypes.

Argument marshalling only: every step of the factorisations and solves runs in
the HIP kernels of libfastfact.so.  PyTorch supplies device memory (tensors)
and streams.  There is no fallback: if the library is missing, loading raises.

Matrix convention: a matrix argument is a 2-D torch tensor M whose logical
element (i, j) is M[i, j] and whose memory is column-major, i.e.
M.stride(0) == 1 and M.stride(1) = ld >= rows (e.g. a Fortran-ordered numpy
array moved with torch.from_numpy(a).to(device), or t.t() of a contiguous
row-major tensor t).
"""
from __future__ import annotations

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfastfact.so")

F64, F32, BF16 = 0, 1, 2
FLAG_STRASSEN1 = 1
FLAG_NO_LOOKAHEAD = 2
FLAG_FIXED_STEP = 4
FLAG_ESCALATE = 8
FLAG_GMRES_IR = 16
FLAG_STRASSEN2 = 32
ERR_HIP, ERR_WORKSPACE, ERR_UNSUPPORTED, ERR_SCRATCH = -100, -101, -102, -103

_DTYPES = {"f64": F64, "f32": F32, "bf16": BF16, F64: F64, F32: F32, BF16: BF16}
_STORAGE = {F64: torch.float64, F32: torch.float32, BF16: torch.float32}

# Every symbol include/fastfact.h declares.
EXPORTED = (
    "ff_status_string", "ff_version", "ff_chol_workspace_size", "chol_factor",
    "ff_lu_workspace_size", "lu_nopiv_factor", "ff_qr_workspace_size", "ff_qr_step", "qr_factor",
    "ff_solve_workspace_size", "chol_solve",
    "ff_trisolve_workspace_size", "chol_trisolve", "chol_trisolve_noalloc", "ff_update_syrk", "ff_update_gemm",
    "ff_update_profile_enable", "ff_update_profile_read",
    "ff_server_create", "ff_server_destroy", "ff_server_submit", "ff_server_step", "ff_server_poll",
    "ff_server_get_stats",
)

UPD_SHAPES = ("64x64", "128x128", "256x128", "f32", "bf16")   # FF_UPD_SHAPE_* order


class ServerResult(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("info", ctypes.c_int32), ("cache_hit", ctypes.c_int32),
                ("latency_ms", ctypes.c_double), ("iters", ctypes.c_int32), ("converged", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("submitted", "completed", "steps", "grouped_launches", "cache_hits",
                                              "evictions", "arena_free", "resident_factors", "queued", "active")]


class KernelProfile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("total_ms", ctypes.c_double), ("total_flops", ctypes.c_double),
                ("total_bytes", ctypes.c_double)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("info", ctypes.c_int32), ("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("dtype_used", ctypes.c_int32), ("last_correction", ctypes.c_double),
                ("backward_err", ctypes.c_double), ("escalated_to", ctypes.c_int32),
                ("escalations", ctypes.c_int32), ("total_iters", ctypes.c_int32), ("first_info", ctypes.c_int32),
                ("krylov_iters", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class FastFactError(RuntimeError):
    pass


_lib = None


def load():
    """Load libfastfact.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FastFactError(f"{LIB_PATH} is missing: build it with `python -m paper_1812_02056_amd.build` "
                            "(there is no non-HIP fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    i64, u32, i32, vp, sz, dbl = (ctypes.c_int64, ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p,
                                  ctypes.c_size_t, ctypes.c_double)
    lib.ff_status_string.argtypes = [i32]
    lib.ff_status_string.restype = ctypes.c_char_p
    lib.ff_version.argtypes = []
    lib.ff_version.restype = ctypes.c_char_p
    lib.ff_chol_workspace_size.argtypes = [i64, i64, i32, u32]
    lib.ff_chol_workspace_size.restype = sz
    lib.chol_factor.argtypes = [i64, i64, vp, i64, i32, u32, vp, sz, vp, vp]
    lib.chol_factor.restype = i32
    lib.ff_lu_workspace_size.argtypes = [i64, i64, i32, u32]
    lib.ff_lu_workspace_size.restype = sz
    lib.lu_nopiv_factor.argtypes = [i64, i64, vp, i64, i32, u32, vp, sz, vp, vp]
    lib.lu_nopiv_factor.restype = i32
    lib.ff_qr_workspace_size.argtypes = [i64, i64, i64, i32, u32]
    lib.ff_qr_workspace_size.restype = sz
    lib.ff_qr_step.argtypes = [i64, i64, i64]
    lib.ff_qr_step.restype = i32
    lib.qr_factor.argtypes = [i64, i64, i64, vp, i64, vp, i64, vp, i64, i32, u32, vp, sz, vp, vp]
    lib.qr_factor.restype = i32
    lib.ff_solve_workspace_size.argtypes = [i64, i64, i64, i32, u32]
    lib.ff_solve_workspace_size.restype = sz
    lib.chol_solve.argtypes = [i64, i64, i64, vp, i64, vp, i64, i32, u32, i32, vp, i64, vp, i64,
                               dbl, i32, vp, sz, vp, ctypes.POINTER(SolveInfo)]
    lib.chol_solve.restype = i32
    lib.ff_trisolve_workspace_size.argtypes = [i64, i32]
    lib.ff_trisolve_workspace_size.restype = sz
    lib.chol_trisolve.argtypes = [i64, i64, vp, i64, i32, vp, i64, vp, sz, vp]
    lib.chol_trisolve.restype = i32
    lib.chol_trisolve_noalloc.argtypes = [i64, i64, vp, i64, i32, vp, i64, vp, vp]
    lib.chol_trisolve_noalloc.restype = i32
    lib.ff_update_syrk.argtypes = [i64, i64, vp, i64, vp, i64, i32, u32, vp]
    lib.ff_update_syrk.restype = i32
    lib.ff_update_gemm.argtypes = [i64, i64, vp, i64, vp, i64, vp, i64, i32, u32, vp]
    lib.ff_update_gemm.restype = i32
    lib.ff_update_profile_enable.argtypes = [i32]
    lib.ff_update_profile_enable.restype = i32
    lib.ff_update_profile_read.argtypes = [ctypes.POINTER(KernelProfile)]
    lib.ff_update_profile_read.restype = i32
    lib.ff_server_create.argtypes = [vp, sz, i32, vp, ctypes.POINTER(i32)]
    lib.ff_server_create.restype = vp
    lib.ff_server_destroy.argtypes = [vp]
    lib.ff_server_destroy.restype = i32
    lib.ff_server_submit.argtypes = [vp, ctypes.c_uint64, i64, vp, i64, vp, i64, i64, vp, i64,
                                     ctypes.POINTER(i64)]
    lib.ff_server_submit.restype = i32
    lib.ff_server_step.argtypes = [vp]
    lib.ff_server_step.restype = i32
    lib.ff_server_poll.argtypes = [vp, ctypes.POINTER(ServerResult), i32, ctypes.POINTER(i32)]
    lib.ff_server_poll.restype = i32
    lib.ff_server_get_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    lib.ff_server_get_stats.restype = i32
    _lib = lib
    return lib


def status_string(code: int) -> str:
    return load().ff_status_string(int(code)).decode()


def version() -> str:
    return load().ff_version().decode()


def _check(rc: int, what: str):
    if rc != 0:
        raise FastFactError(f"{what} failed: {rc} ({status_string(rc)})")


def _dt(dtype) -> int:
    try:
        return _DTYPES[dtype]
    except KeyError:
        raise ValueError(f"unknown dtype {dtype!r}") from None


def _ld(M: torch.Tensor, name: str) -> int:
    if M.dim() != 2:
        raise ValueError(f"{name} must be 2-D")
    if M.shape[0] > 1 and M.stride(0) != 1:
        raise ValueError(f"{name} must be column-major (stride(0) == 1)")
    return max(int(M.stride(1)) if M.shape[1] > 1 else int(M.shape[0]), int(M.shape[0]), 1)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def colmajor_empty(rows: int, cols: int, dtype, device, ld: int | None = None) -> torch.Tensor:
    """An uninitialised rows x cols column-major tensor with leading dimension ld."""
    ld = rows if ld is None else ld
    return torch.empty((cols, ld), dtype=dtype, device=device).t()[:rows]


def to_device(a, device="cuda", dtype=None, ld: int | None = None) -> torch.Tensor:
    """Copy a (numpy or torch) matrix to a column-major device tensor."""
    t = torch.as_tensor(a)
    if t.dim() == 1:
        t = t.reshape(-1, 1)
    dt = dtype or t.dtype
    out = colmajor_empty(t.shape[0], t.shape[1], dt, device, ld)
    out.copy_(t.to(dt))
    return out


def _workspace(nbytes: int, device) -> torch.Tensor | None:
    if nbytes == 0:
        return None
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device)


def chol_workspace_size(n: int, s: int, dtype="f64", strassen=False) -> int:
    return int(load().ff_chol_workspace_size(n, s, _dt(dtype), FLAG_STRASSEN1 if strassen else 0))


def chol_factor(A: torch.Tensor, s: int, dtype="f64", strassen=False, no_lookahead=False, stream=None,
                ws: torch.Tensor | None = None, info: torch.Tensor | None = None, sync=False, fixed_step=False):
    """In-place Cholesky A = L L^T (tril(A) read and overwritten).  Returns the
    device int32 info tensor, or (sync=True) its value as a Python int.
    fixed_step: every block exactly s wide (FF_FLAG_FIXED_STEP)."""
    lib = load()
    dt = _dt(dtype)
    n = int(A.shape[0])
    if A.shape[1] != n:
        raise ValueError("A must be square")
    if A.dtype != _STORAGE[dt]:
        raise ValueError(f"A must be {_STORAGE[dt]} for dtype {dtype}")
    flags = ((FLAG_STRASSEN1 if strassen else 0) | (FLAG_NO_LOOKAHEAD if no_lookahead else 0)
             | (FLAG_FIXED_STEP if fixed_step else 0))
    need = int(lib.ff_chol_workspace_size(n, s, dt, flags))
    if ws is None:
        ws = _workspace(need, A.device)
    if info is None:
        info = torch.empty(1, dtype=torch.int32, device=A.device)
    rc = lib.chol_factor(n, s, _ptr(A), _ld(A, "A"), dt, flags, _ptr(ws), 0 if ws is None else ws.numel(),
                         _ptr(info), _stream(stream))
    _check(rc, "chol_factor")
    if sync:
        (stream or torch.cuda.current_stream()).synchronize()
        return int(info.item())
    return info


def lu_nopiv_factor(A: torch.Tensor, s: int, dtype="f64", strassen=False, no_lookahead=False, stream=None,
                    info: torch.Tensor | None = None, sync=False, fixed_step=False, ws: torch.Tensor | None = None):
    """In-place LU without pivoting, Doolittle packed (unit-lower L below the diagonal, U on and above).
    strassen: False, True / 1 (one level, FF_FLAG_STRASSEN1) or 2 (two levels, FF_FLAG_STRASSEN2).
    fixed_step: every block exactly s wide (FF_FLAG_FIXED_STEP)."""
    lib = load()
    dt = _dt(dtype)
    n = int(A.shape[0])
    if A.shape[1] != n:
        raise ValueError("A must be square")
    levels = int(strassen)
    flags = ((FLAG_STRASSEN1 if levels == 1 else FLAG_STRASSEN2 if levels == 2 else 0)
             | (FLAG_NO_LOOKAHEAD if no_lookahead else 0) | (FLAG_FIXED_STEP if fixed_step else 0))
    need = int(lib.ff_lu_workspace_size(n, s, dt, flags))
    if ws is None:
        ws = _workspace(need, A.device)
    if info is None:
        info = torch.empty(1, dtype=torch.int32, device=A.device)
    rc = lib.lu_nopiv_factor(n, s, _ptr(A), _ld(A, "A"), dt, flags, _ptr(ws), 0 if ws is None else ws.numel(),
                             _ptr(info), _stream(stream))
    _check(rc, "lu_nopiv_factor")
    if sync:
        (stream or torch.cuda.current_stream()).synchronize()
        return int(info.item())
    return info


def qr_workspace_size(m: int, n: int, s: int, dtype="f64") -> int:
    return int(load().ff_qr_workspace_size(m, n, s, _dt(dtype), 0))


def qr_step(m: int, n: int, s: int) -> int:
    """The block width qr_factor uses for step s (bounded by the Gram-Schmidt
    kernel's LDS-resident block)."""
    return int(load().ff_qr_step(m, n, s))


def qr_factor(A: torch.Tensor, s: int, Q: torch.Tensor | None = None, R: torch.Tensor | None = None,
              dtype="f64", stream=None, ws: torch.Tensor | None = None, info: torch.Tensor | None = None,
              sync=False):
    """A = Q R (A m x n column-major, m >= n, read only).  Returns (Q, R, info);
    info is an int when sync, else the device tensor."""
    lib = load()
    dt = _dt(dtype)
    m, n = int(A.shape[0]), int(A.shape[1])
    if Q is None:
        Q = colmajor_empty(m, n, A.dtype, A.device)
    if R is None:
        R = colmajor_empty(n, n, A.dtype, A.device)
    if ws is None:
        ws = _workspace(int(lib.ff_qr_workspace_size(m, n, s, dt, 0)), A.device)
    if info is None:
        info = torch.zeros(1, dtype=torch.int32, device=A.device)
    rc = lib.qr_factor(m, n, s, _ptr(A), _ld(A, "A"), _ptr(Q), _ld(Q, "Q"), _ptr(R), _ld(R, "R"), dt, 0,
                       _ptr(ws), 0 if ws is None else ws.numel(), _ptr(info), _stream(stream))
    _check(rc, "qr_factor")
    if sync:
        (stream or torch.cuda.current_stream()).synchronize()
        return Q, R, int(info.item())
    return Q, R, info


def solve_workspace_size(n: int, s: int, nrhs: int, dtype="f64", escalate=False, gmres=False) -> int:
    flags = (FLAG_ESCALATE if escalate else 0) | (FLAG_GMRES_IR if gmres else 0)
    return int(load().ff_solve_workspace_size(n, s, nrhs, _dt(dtype), flags))


def chol_solve(A64: torch.Tensor, B: torch.Tensor, s: int, dtype="f32", W: torch.Tensor | None = None,
               w_is_factored=False, X: torch.Tensor | None = None, tol=1e-13, max_iter=50, strassen=False,
               stream=None, ws: torch.Tensor | None = None, escalate=False, no_lookahead=False, gmres=False):
    """Solve A64 X = B with a factor W in `dtype` and binary64 refinement
    (escalate: refactor in higher precision when that fails, FF_FLAG_ESCALATE;
    gmres: correction equations solved by factor-preconditioned GMRES,
    FF_FLAG_GMRES_IR).
    Returns (X, W, info dict).  Synchronises the stream."""
    lib = load()
    dt = _dt(dtype)
    n = int(A64.shape[0])
    nrhs = int(B.shape[1])
    flags = ((FLAG_STRASSEN1 if strassen else 0) | (FLAG_ESCALATE if escalate else 0)
             | (FLAG_NO_LOOKAHEAD if no_lookahead else 0) | (FLAG_GMRES_IR if gmres else 0))
    if W is None:
        if w_is_factored:
            raise ValueError("w_is_factored requires W")
        W = colmajor_empty(n, n, _STORAGE[dt], A64.device)
    if X is None:
        X = colmajor_empty(n, nrhs, torch.float64, A64.device)
    if ws is None:
        ws = _workspace(int(lib.ff_solve_workspace_size(n, s, nrhs, dt, flags)), A64.device)
    out = SolveInfo()
    rc = lib.chol_solve(n, s, nrhs, _ptr(A64), _ld(A64, "A64"), _ptr(W), _ld(W, "W"), dt, flags,
                        1 if w_is_factored else 0, _ptr(B), _ld(B, "B"), _ptr(X), _ld(X, "X"), float(tol),
                        int(max_iter), _ptr(ws), 0 if ws is None else ws.numel(), _stream(stream), ctypes.byref(out))
    _check(rc, "chol_solve")
    return X, W, out.as_dict()


def trisolve_workspace_size(n: int, dtype="f64") -> int:
    return int(load().ff_trisolve_workspace_size(n, _dt(dtype)))


def chol_trisolve(L: torch.Tensor, X: torch.Tensor, dtype="f64", stream=None, ws: torch.Tensor | None = None):
    """X <- L^-T L^-1 X in place, in L's storage precision.  The first int32 of
    the workspace is the error word (nonzero if a bounded wait expired)."""
    lib = load()
    dt = _dt(dtype)
    n = int(L.shape[0])
    if ws is None:
        ws = _workspace(int(lib.ff_trisolve_workspace_size(n, dt)), L.device)
    rc = lib.chol_trisolve(n, int(X.shape[1]), _ptr(L), _ld(L, "L"), dt, _ptr(X), _ld(X, "X"),
                           _ptr(ws), 0 if ws is None else ws.numel(), _stream(stream))
    _check(rc, "chol_trisolve")
    return X


def chol_trisolve_noalloc(L: torch.Tensor, X: torch.Tensor, dtype="f64", status: torch.Tensor | None = None,
                          stream=None):
    """chol_trisolve with the library's static device scratch (no allocation
    anywhere).  status: optional device int32 tensor receiving the error word."""
    rc = load().chol_trisolve_noalloc(int(L.shape[0]), int(X.shape[1]), _ptr(L), _ld(L, "L"), _dt(dtype), _ptr(X),
                                      _ld(X, "X"), _ptr(status), _stream(stream))
    _check(rc, "chol_trisolve_noalloc")
    return X


def update_syrk(C: torch.Tensor, P: torch.Tensor, dtype="f64", strassen=False, stream=None):
    """tril(C) -= tril(P P^T) (Algorithm 1's deferred update) in place."""
    rc = load().ff_update_syrk(int(C.shape[0]), int(P.shape[1]), _ptr(C), _ld(C, "C"), _ptr(P), _ld(P, "P"),
                               _dt(dtype), FLAG_STRASSEN1 if strassen else 0, _stream(stream))
    _check(rc, "ff_update_syrk")
    return C


def update_gemm(C: torch.Tensor, X: torch.Tensor, Y: torch.Tensor, dtype="f64", strassen=False, stream=None):
    """C -= X Y (Algorithm 2's deferred update) in place."""
    rc = load().ff_update_gemm(int(C.shape[0]), int(X.shape[1]), _ptr(C), _ld(C, "C"), _ptr(X), _ld(X, "X"),
                               _ptr(Y), _ld(Y, "Y"), _dt(dtype), FLAG_STRASSEN1 if strassen else 0,
                               _stream(stream))
    _check(rc, "ff_update_gemm")
    return C


def update_profile_enable(enable: bool = True):
    """Start (clearing the tallies) or stop event timing of chol_factor's trailing updates."""
    _check(load().ff_update_profile_enable(1 if enable else 0), "ff_update_profile_enable")


def update_profile_read() -> dict:
    """Per kernel shape: launches, total_ms, total_flops, total_bytes (algorithmic)
    since the last enable (synchronises)."""
    out = (KernelProfile * len(UPD_SHAPES))()
    _check(load().ff_update_profile_read(out), "ff_update_profile_read")
    return {UPD_SHAPES[i]: {"launches": int(out[i].launches), "total_ms": float(out[i].total_ms),
                            "total_flops": float(out[i].total_flops), "total_bytes": float(out[i].total_bytes)}
            for i in range(len(UPD_SHAPES))}


class Server:
    """Continuous-batching solver (ff_server_*): many independent SPD systems
    (binary64 A, B, X), every admitted factorisation advanced one block per
    step() with grouped launches; finished factors stay resident under their
    key.  dtype "f64": binary64 factors; "f32": binary32 factors with binary64
    refinement.

    arena: a device tensor whose storage is the HBM budget (kept alive here).
    Tensors passed to submit() are kept alive until their request is polled."""

    def __init__(self, arena: torch.Tensor, stream=None, dtype="f64"):
        self._lib = load()
        self.arena = arena
        self.stream = stream if stream is not None else torch.cuda.current_stream(arena.device)
        st = ctypes.c_int(0)
        h = self._lib.ff_server_create(_ptr(arena), arena.numel() * arena.element_size(), _dt(dtype),
                                       _stream(self.stream), ctypes.byref(st))
        if not h:
            raise FastFactError(f"ff_server_create failed: {st.value} ({status_string(st.value)})")
        self._h = ctypes.c_void_p(h)
        self._keep = {}

    def submit(self, A: torch.Tensor, B: torch.Tensor, X: torch.Tensor, key: int = 0) -> int:
        """A: n x n column-major float64 (lower triangle read); B, X: n x nrhs column-major."""
        n = int(A.shape[0])
        for name, T in (("A", A), ("B", B), ("X", X)):
            if T.dtype != torch.float64 or not T.is_cuda:
                raise ValueError(f"{name} must be a float64 device tensor")
        if A.shape[1] != n or B.shape[0] != n or tuple(X.shape) != tuple(B.shape):
            raise ValueError("A must be n x n and B, X n x nrhs")
        rid = ctypes.c_int64(0)
        rc = self._lib.ff_server_submit(self._h, int(key), n, _ptr(A), _ld(A, "A"), _ptr(B), int(B.shape[1]),
                                        _ld(B, "B"), _ptr(X), _ld(X, "X"), ctypes.byref(rid))
        _check(rc, "ff_server_submit")
        self._keep[rid.value] = (A, B, X)
        return rid.value

    def step(self) -> int:
        rc = self._lib.ff_server_step(self._h)
        if rc < 0:
            _check(rc, "ff_server_step")
        return rc

    def poll(self, max_out: int = 256) -> list:
        out = (ServerResult * max_out)()
        k = ctypes.c_int(0)
        _check(self._lib.ff_server_poll(self._h, out, max_out, ctypes.byref(k)), "ff_server_poll")
        res = []
        for i in range(k.value):
            r = out[i]
            self._keep.pop(r.id, None)
            res.append({"id": r.id, "info": r.info, "cache_hit": bool(r.cache_hit), "latency_ms": r.latency_ms,
                        "iters": r.iters, "converged": bool(r.converged)})
        return res

    def stats(self) -> dict:
        st = ServerStats()
        _check(self._lib.ff_server_get_stats(self._h, ctypes.byref(st)), "ff_server_get_stats")
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ff_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
