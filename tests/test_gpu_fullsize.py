"""Full-size GPU checks at n = 16384, in the configuration bench.py times (binary64,
lookahead schedule, the benchmark's step sizes):

* the benchmark matrices against the CPU oracle, element by element: Cholesky of
  A = G G^T / n + I (kappa ~ 5) at the paper's step s = 168 and at the benchmark's
  s = 768 with ||tril(L - L_oracle)||_F / ||tril(L)||_F <= 1e-11; LU without
  pivoting of the strictly diagonally dominant U(-1, 1) matrix at s = 168 against
  the oracle's Doolittle factors at the same bound, backward error <= 1e-13
  (the oracle runs on all host cores: about half a minute for Cholesky and a
  minute for LU);

* integer families: A = L0 L0^T (or L0 U0) formed by torch's binary64 GEMM, exact
  for these entries; the factor must equal L0 (U0) bit for bit, as at small sizes,
  with the classical and with the one-level Strassen update;
* the benchmark matrix A = G G^T / n + I: backward error by torch's GEMM, and
  sampled entries of L L^T recomputed on the host in binary64 from the factor's
  rows against A;
* refined solves: an integer solution x0 recovered from b = A x0 (A the benchmark
  family).
"""
import numpy as np
import pytest

import oracle
from paper_1812_02056_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1812_02056_amd as ff  # noqa: E402

DEV = torch.device("cuda:0")
N = 16384


def colmajor(A_rowmajor):
    out = torch.empty_strided(A_rowmajor.shape, (1, A_rowmajor.shape[0]), dtype=A_rowmajor.dtype, device=DEV)
    out.copy_(A_rowmajor)
    return out


@pytest.mark.parametrize("s", [256, 168])
def test_fullsize_chol_integer_family_bitwise(s):
    L0, A = wl.chol_int_family_device(N, seed=5, device=DEV)
    Acm = A.t()                                  # symmetric: the same storage read column-major
    assert ff.chol_factor(Acm, s, dtype="f64", sync=True) == 0
    assert torch.equal(torch.tril(Acm), L0)
    del L0, A, Acm
    torch.cuda.empty_cache()


@pytest.mark.parametrize("s", [384, 640, 768])
@pytest.mark.parametrize("fixed_step", [False, True])
def test_fullsize_chol_integer_family_bitwise_wide_steps(s, fixed_step):
    # the benchmark's steps; by default the first block and the last 6144 columns
    # are 192-wide blocks, with fixed_step every block is s wide
    L0, A = wl.chol_int_family_device(N, seed=9, device=DEV)
    Acm = A.t()
    assert ff.chol_factor(Acm, s, dtype="f64", fixed_step=fixed_step, sync=True) == 0
    assert torch.equal(torch.tril(Acm), L0)
    del L0, A, Acm
    torch.cuda.empty_cache()


def test_fullsize_chol_benchmark_matrix():
    s = 256
    A0 = wl.spd_scaled_device(N, seed=0, device=DEV)
    Acm = A0.clone().t()
    assert ff.chol_factor(Acm, s, dtype="f64", sync=True) == 0
    L = torch.tril(Acm)
    bwd = float(torch.linalg.norm(A0.t() - L @ L.t().contiguous()) / torch.linalg.norm(A0))
    assert bwd <= 1e-13
    # sampled entries of L L^T against A, summed on the host in binary64
    rng = np.random.default_rng(11)
    idx = np.unique(np.concatenate([rng.integers(0, N, 40), [0, 1, N - 1, N - 2]]))
    rows = L[idx].cpu().numpy()                  # the factor's rows i (L(i, :))
    Ah = A0[idx][:, idx].cpu().numpy()
    for a, i in enumerate(idx):
        for b, j in enumerate(idx):
            if j > i:
                continue
            k = min(i, j) + 1
            v = float(np.dot(rows[a, :k], rows[b, :k]))
            assert abs(v - Ah[a, b]) <= 1e-13 * max(1.0, abs(Ah[a, b])) * 4, (i, j)
    del A0, Acm, L
    torch.cuda.empty_cache()


@pytest.mark.parametrize("s", [168, 768])
def test_fullsize_lu_integer_family_bitwise(s):
    L0, U0, A = wl.lu_int_family_device(N, seed=6, device=DEV)
    Acm = colmajor(A)
    del A
    assert ff.lu_nopiv_factor(Acm, s, sync=True) == 0
    assert torch.equal(torch.tril(Acm, -1), torch.tril(L0, -1))
    assert torch.equal(torch.triu(Acm), U0)
    del L0, U0, Acm
    torch.cuda.empty_cache()


@pytest.mark.parametrize("s", [320, 512])
def test_fullsize_chol_strassen_integer_family_bitwise(s):
    # one Strassen level in every trailing update (lookahead schedule): operand sums
    # and products stay small integers, so the factor is L0 bit for bit
    L0, A = wl.chol_int_family_device(N, seed=9, device=DEV)
    Acm = A.t()
    assert ff.chol_factor(Acm, s, dtype="f64", strassen=True, sync=True) == 0
    assert torch.equal(torch.tril(Acm), L0)
    del L0, A, Acm
    torch.cuda.empty_cache()


def test_fullsize_lu_strassen_integer_family_bitwise():
    L0, U0, A = wl.lu_int_family_device(N, seed=10, device=DEV)
    Acm = colmajor(A)
    del A
    assert ff.lu_nopiv_factor(Acm, 168, strassen=True, sync=True) == 0
    assert torch.equal(torch.tril(Acm, -1), torch.tril(L0, -1))
    assert torch.equal(torch.triu(Acm), U0)
    del L0, U0, Acm
    torch.cuda.empty_cache()


@pytest.mark.parametrize("s", [320, 640, 768])
def test_fullsize_chol_benchmark_matrix_wide_steps(s):
    # the step sizes the benchmark's sweep picks between: backward error of the
    # timed configuration
    A0 = wl.spd_scaled_device(N, seed=0, device=DEV)
    Acm = A0.clone().t()
    assert ff.chol_factor(Acm, s, dtype="f64", sync=True) == 0
    L = torch.tril(Acm)
    bwd = float(torch.linalg.norm(A0.t() - L @ L.t().contiguous()) / torch.linalg.norm(A0))
    assert bwd <= 1e-13
    del A0, Acm, L
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype,s", [("f64", 256), ("f32", 256), ("bf16", 512), ("f64", 640), ("f32", 640),
                                     ("bf16", 768)])
def test_fullsize_refined_solve_integer_solution(dtype, s):
    # the benchmark family (kappa ~ 5); b = A x0 by torch's GEMM, so x0 is recovered
    # to about kappa * 1e-16 (the integer family's triangular factors are too
    # ill-conditioned to solve with at this size, though they factor exactly)
    A = wl.spd_scaled_device(N, seed=3, device=DEV)
    x0 = torch.randint(-1, 2, (2, N), generator=torch.Generator().manual_seed(8)).to(DEV, torch.float64)
    B = (A @ x0.t().contiguous()).t().contiguous().t()        # column-major n x 2
    X, W, info = ff.chol_solve(A.t(), B, s, dtype=dtype, tol=1e-13, max_iter=50)
    assert info["info"] == 0
    if dtype != "f64":
        assert info["converged"] == 1
    assert float((X - x0.t()).abs().max()) <= 1e-12
    assert info["backward_err"] <= 1e-15
    del A, B, X, W
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def benchmark_chol_oracle():
    A0 = wl.spd_scaled_device(N, seed=0, device=DEV)     # the benchmark's matrix (symmetric, row-major)
    Lo, info = oracle.chol(A0.cpu().numpy())
    assert info == 0
    return A0, Lo


@pytest.mark.parametrize("s", [168, 768])
def test_fullsize_chol_benchmark_matrix_matches_oracle(benchmark_chol_oracle, s):
    A0, Lo = benchmark_chol_oracle
    Acm = A0.clone().t()
    assert ff.chol_factor(Acm, s, dtype="f64", sync=True) == 0
    L = torch.tril(Acm).cpu().numpy()
    del Acm
    torch.cuda.empty_cache()
    rel = oracle.rel_lower(L, Lo)
    print(f"n={N} s={s}: rel_L = {rel:.2e}")
    assert rel <= 1e-11


def test_fullsize_lu_matches_oracle():
    s = 168
    T = wl.diag_dominant_device(N, seed=0, device=DEV)   # T[j, i] = A[i, j]: column-major storage of A
    A_host = T.t().cpu().numpy()
    LUo, info = oracle.lu(A_host)
    assert info == 0
    Acm = T.clone().t()
    assert ff.lu_nopiv_factor(Acm, s, sync=True) == 0
    LU = Acm.cpu().numpy()
    d = LU - LUo
    rel = float(np.linalg.norm(d) / np.linalg.norm(LUo))
    del d
    # backward error with torch's binary64 GEMM on the device (independent of the library's kernels)
    Ld = torch.tril(Acm, -1)
    Ld.diagonal().fill_(1.0)
    Ud = torch.triu(Acm)
    bwd = float(torch.linalg.norm(T.t() - Ld @ Ud) / torch.linalg.norm(T))
    print(f"LU n={N} s={s}: rel = {rel:.2e} bwd = {bwd:.2e}")
    del T, Acm, Ld, Ud
    torch.cuda.empty_cache()
    assert rel <= 1e-11
    assert bwd <= 1e-13
