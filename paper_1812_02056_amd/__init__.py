"""Delayed-update Cholesky / LU for AMD MI355X (gfx950).

The method is C. Camarero, arXiv 1812.02056 (Sec. 2, Algorithms 1, 2 and 3).  The
computation runs in the HIP kernels of libfastfact.so (C ABI in
include/fastfact.h); `binding` marshals torch tensors to it.  The API names are
the C entry points: chol_factor, lu_nopiv_factor, qr_factor, chol_solve, chol_trisolve,
update_syrk, update_gemm.
"""
_API = ("chol_factor", "lu_nopiv_factor", "qr_factor", "qr_workspace_size", "qr_step", "chol_solve", "chol_trisolve", "chol_trisolve_noalloc", "update_syrk", "update_gemm",
        "chol_workspace_size", "solve_workspace_size", "trisolve_workspace_size", "status_string", "version", "to_device",
        "colmajor_empty", "FastFactError", "load", "update_profile_enable", "update_profile_read", "Server")


def __getattr__(name):
    if name in _API:
        from . import binding
        return getattr(binding, name)
    raise AttributeError(name)
