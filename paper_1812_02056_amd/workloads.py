"""Seeded synthetic inputs for the Cholesky / LU library, its tests and its benchmark.

This module only draws random matrices and right-hand sides; it holds none of
the factorisation arithmetic, so both the GPU path and the CPU oracle can take
their inputs from it.  Every generator is deterministic in ``seed``.

The paper times its method on a random symmetric matrix whose diagonal is made
large (Sec. 2, the timing paragraph after the cost analysis) and does not say
how the entries are drawn; the families here are concrete stand-ins with known
conditioning:

* ``spd_shifted``  A = G G^T + n I            (G i.i.d. N(0,1); kappa ~ 5)
* ``spd_scaled``   A = G G^T / n + lam I      (kappa ~ 5 / 4e3 / 2e6 for lam = 1 / 1e-3 / 1e-6)
* ``chol_int_family``  A = L0 L0^T with L0 integer, diag in {1,2}, off-diagonal in
  {-1,0,1}: every intermediate of any evaluation order is a small integer, so the
  factor must come out as L0 bit for bit.
* ``chol_float_family``  A = L0 L0^T with off-diagonal N(0, 1/n) (or N(0,1)), diag U(1,2).
* ``lu_int_family``  A = L0 U0, L0 unit lower and U0 upper with diag in {1,2},
  off-diagonal entries in {-1,0,1}.
* ``diag_dominant``  U(-1,1) entries, diagonal 1 + row sum of |off-diagonal|.
* ``qr_int_family``  A = Q0 R0 with Q0 = H[:, :n] / sqrt(m) (H the m x m Sylvester
  Hadamard matrix, m a power of 4 so sqrt(m) is a power of two) and R0 = sqrt(m) U,
  U upper triangular with diagonal in {1,2} and entries in {-1,0,1} above it:
  every value Gram-Schmidt forms is a dyadic rational of modest size, so Q and R
  must come out as Q0 and R0 bit for bit.

All matrices are returned column-major (numpy order='F') float64.  Symmetric
families are mirrored lower -> upper after forming, so they are bitwise symmetric.
"""
from __future__ import annotations

import numpy as np


def _mirror_lower(A: np.ndarray) -> np.ndarray:
    L = np.tril(A)
    return np.asfortranarray(L + np.tril(A, -1).T)


def spd_shifted(n: int, seed: int = 0) -> np.ndarray:
    """A = G G^T + n I, G n x n i.i.d. N(0,1)."""
    g = np.random.default_rng(seed).standard_normal((n, n))
    A = g @ g.T
    A[np.diag_indices(n)] += float(n)
    return _mirror_lower(A)


def spd_scaled(n: int, seed: int = 0, lam: float = 1.0) -> np.ndarray:
    """A = G G^T / n + lam I, G n x n i.i.d. N(0,1)."""
    g = np.random.default_rng(seed).standard_normal((n, n))
    A = (g @ g.T) / float(n)
    A[np.diag_indices(n)] += float(lam)
    return _mirror_lower(A)


def chol_int_family(n: int, seed: int = 0, p_zero: float = 1.0 / 3.0):
    """(L0, A) with A = L0 L0^T exactly; L0 lower, diag in {1,2}, off-diag in {-1,0,1}."""
    rng = np.random.default_rng(seed)
    p_nz = (1.0 - p_zero) / 2.0
    off = rng.choice(np.array([-1, 0, 1], dtype=np.int64), size=(n, n), p=[p_nz, p_zero, p_nz])
    L0 = np.tril(off, -1)
    L0[np.diag_indices(n)] = rng.integers(1, 3, size=n)
    L0f = L0.astype(np.float64)
    A = L0f @ L0f.T                                # integer partial sums of magnitude <= 4n: exact in binary64
    return np.asfortranarray(L0f), np.asfortranarray(A)


def chol_float_family(n: int, seed: int = 0, scaled: bool = True):
    """(L0, A) with A = fl(L0 L0^T); off-diagonal N(0, 1/n) if scaled else N(0,1); diag U(1,2)."""
    rng = np.random.default_rng(seed)
    off = rng.standard_normal((n, n))
    if scaled:
        off /= np.sqrt(float(n))
    L0 = np.tril(off, -1)
    L0[np.diag_indices(n)] = rng.uniform(1.0, 2.0, size=n)
    A = L0 @ L0.T
    return np.asfortranarray(L0), _mirror_lower(A)


def lu_int_family(n: int, seed: int = 0):
    """(L0, U0, A): A = L0 U0 exactly; L0 unit lower, U0 upper, diag(U0) in {1,2}."""
    rng = np.random.default_rng(seed)
    vals = np.array([-1, 0, 1], dtype=np.int64)
    L0 = np.tril(rng.choice(vals, size=(n, n)), -1) + np.eye(n, dtype=np.int64)
    U0 = np.triu(rng.choice(vals, size=(n, n)), 1)
    U0[np.diag_indices(n)] = rng.integers(1, 3, size=n)
    L0f, U0f = L0.astype(np.float64), U0.astype(np.float64)
    A = L0f @ U0f              # integer partial sums of magnitude <= 2n: exact in binary64
    return np.asfortranarray(L0f), np.asfortranarray(U0f), np.asfortranarray(A)


def diag_dominant(n: int, seed: int = 0) -> np.ndarray:
    """U(-1,1) entries with A[i,i] = 1 + sum_{j != i} |A[i,j]| (strict row dominance)."""
    A = np.random.default_rng(seed).uniform(-1.0, 1.0, size=(n, n))
    A[np.diag_indices(n)] = 0.0
    A[np.diag_indices(n)] = 1.0 + np.sum(np.abs(A), axis=1)
    return np.asfortranarray(A)


def rhs(n: int, nrhs: int = 1, seed: int = 0) -> np.ndarray:
    """n x nrhs i.i.d. N(0,1) right-hand sides."""
    return np.asfortranarray(np.random.default_rng(seed).standard_normal((n, nrhs)))


def default_s(n: int) -> int:
    """Step size s = round(n^0.5286), the exponent the paper's complexity analysis
    arrives at with Le Gall-Urrutia rectangular multiplication (Sec. 2, cost discussion)."""
    return max(1, int(round(float(n) ** 0.5286)))


def hadamard(m: int) -> np.ndarray:
    """Sylvester Hadamard matrix of order m (a power of two), entries +-1."""
    if m < 1 or m & (m - 1):
        raise ValueError("m must be a power of two")
    H = np.ones((1, 1))
    while H.shape[0] < m:
        H = np.block([[H, H], [H, -H]])
    return H


def _qr_int_parts(m: int, n: int, seed: int):
    k = int(round(np.log(m) / np.log(4)))
    if 4 ** k != m or n > m:
        raise ValueError("m must be a power of 4 and n <= m")
    rng = np.random.default_rng(seed)
    U = np.triu(rng.integers(-1, 2, size=(n, n)), 1).astype(np.float64)
    U[np.diag_indices(n)] = rng.integers(1, 3, size=n)
    return k, U


def qr_int_family(m: int, n: int, seed: int = 0):
    """(Q0, R0, A): A = H[:, :n] U exactly, Q0 = H[:, :n] / 2^k, R0 = 2^k U (m = 4^k)."""
    k, U = _qr_int_parts(m, n, seed)
    Hn = hadamard(m)[:, :n]
    A = Hn @ U                                      # integers of magnitude <= n + 1: exact
    return (np.asfortranarray(Hn / 2.0 ** k), np.asfortranarray(U * 2.0 ** k), np.asfortranarray(A))


# ---------------------------------------------------------------------------
# Device-side generators for the large configurations (torch; seeded per device).
# The returned tensors hold the matrix in column-major order: element (i, j) at
# offset i + j*n, i.e. the row-major storage of A^T.  For symmetric A they are
# identical to the row-major A.
# ---------------------------------------------------------------------------

def spd_scaled_device(n: int, seed: int = 0, lam: float = 1.0, device="cuda"):
    """A = G G^T / n + lam I on the device (float64), mirrored lower -> upper."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    G = torch.randn(n, n, dtype=torch.float64, device=device, generator=gen)
    A = torch.mm(G, G.t().contiguous())
    del G
    A.div_(float(n))
    A.diagonal().add_(float(lam))
    # mirror: column-major storage of A = row-major storage of A^T; make it exactly symmetric
    A = torch.tril(A) + torch.tril(A, -1).t()
    return A.contiguous()


def diag_dominant_device(n: int, seed: int = 0, device="cuda"):
    """Column-major U(-1,1) matrix with 1 + row-sum-of-|off-diagonal| on the diagonal.

    Returned tensor T satisfies T[j, i] = A[i, j] (T is the row-major view of the
    column-major buffer)."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    A = torch.rand(n, n, dtype=torch.float64, device=device, generator=gen).mul_(2.0).sub_(1.0)
    A.fill_diagonal_(0.0)
    d = A.abs().sum(dim=1).add_(1.0)
    A.diagonal().copy_(d)
    return A.t().contiguous()


def rhs_device(n: int, nrhs: int = 1, seed: int = 0, device="cuda"):
    """Column-major n x nrhs N(0,1) right-hand sides; returned as an (nrhs, n) tensor."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    return torch.randn(nrhs, n, dtype=torch.float64, device=device, generator=gen)


def chol_int_family_device(n: int, seed: int = 0, device="cuda"):
    """(L0, A) on the device, for sizes where the host product is too slow: L0 lower
    with off-diagonal entries uniform on {-1, 0, 1} and diagonal in {1, 2} (drawn on
    the host), A = L0 L0^T formed by a binary64 GEMM, exact because every partial sum
    is an integer of magnitude at most 4n.  Both returned row-major; A is symmetric,
    and L0 read column-major is L0^T."""
    import torch
    rng = np.random.default_rng(seed)
    off = torch.from_numpy(rng.integers(-1, 2, size=(n, n), dtype=np.int8))
    diag = torch.from_numpy(rng.integers(1, 3, size=n, dtype=np.int8))
    L0 = torch.tril(off.to(device=device, dtype=torch.float64), -1)
    del off
    L0.diagonal().copy_(diag.to(device=device, dtype=torch.float64))
    A = torch.mm(L0, L0.t().contiguous())
    return L0, A


def lu_int_family_device(n: int, seed: int = 0, device="cuda"):
    """(L0, U0, A) on the device: L0 unit lower, U0 upper with diagonal in {1, 2},
    off-diagonal entries uniform on {-1, 0, 1}; A = L0 U0 by a binary64 GEMM (exact:
    integer partial sums of magnitude at most 2n).  Row-major tensors."""
    import torch
    rng = np.random.default_rng(seed)
    lo = torch.from_numpy(rng.integers(-1, 2, size=(n, n), dtype=np.int8))
    up = torch.from_numpy(rng.integers(-1, 2, size=(n, n), dtype=np.int8))
    diag = torch.from_numpy(rng.integers(1, 3, size=n, dtype=np.int8))
    L0 = torch.tril(lo.to(device=device, dtype=torch.float64), -1)
    L0.diagonal().fill_(1.0)
    U0 = torch.triu(up.to(device=device, dtype=torch.float64), 1)
    U0.diagonal().copy_(diag.to(device=device, dtype=torch.float64))
    del lo, up
    A = torch.mm(L0, U0)
    return L0, U0, A


def qr_int_family_device(m: int, n: int, seed: int = 0, device="cuda"):
    """(Q0, R0, A) of ``qr_int_family`` as column-major device tensors (stride (1, rows));
    A = H[:, :n] U by a binary64 GEMM, exact (integer partial sums of magnitude <= n + 1)."""
    import torch
    k, U = _qr_int_parts(m, n, seed)
    H = torch.ones(1, 1, dtype=torch.float64, device=device)
    while H.shape[0] < m:
        H = torch.cat([torch.cat([H, H], 1), torch.cat([H, -H], 1)], 0)
    Hn = H[:, :n].contiguous()
    del H
    Ud = torch.from_numpy(U).to(device)
    A = torch.mm(Hn, Ud)

    def cm(t):
        return t.t().contiguous().t()
    return cm(Hn / 2.0 ** k), cm(Ud * 2.0 ** k), cm(A)
