"""QR by Gram-Schmidt with deferred block projections (Sec. 2, Algorithm 3) on the
GPU, against the CPU oracle.

* parity: Q and R element by element against the oracle run with the same block
  width, over square and tall shapes with ragged row counts (not multiples of the
  128-row panel slices) and ragged last blocks, and the special cases s = 1 and
  s >= n.  Bound: the two results are modified-Gram-Schmidt-type QRs of the same
  matrix differing only in rounding order; each is within c n kappa(A) u of the
  exact factors (kappa the 2-norm condition number, u = 2^-53), so the bound on
  |Q - Q_oracle| is 8 n kappa u and on |R - R_oracle| 8 n kappa u max|R|;
* exact family A = H[:, :n] U (every intermediate exact): Q and R bit for bit,
  up to the benchmark's n = 16384;
* the benchmark matrix at n = 16384: orthogonality and residual by torch's
  binary64 GEMM, and the first three blocks of Q and R against the oracle (the
  first c columns of Q and R depend only on the first c columns of A);
* edge cases: a zero and a NaN column (info), n = 0, deterministic results.
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
U = np.finfo(np.float64).eps / 2


def dev(a, ld=None):
    return ff.to_device(a, DEV, ld=ld)


def host(t):
    return t.detach().cpu().numpy()


def matrix(m, n, seed):
    if m == n:
        return wl.spd_scaled(n, seed=seed)              # the benchmark family, kappa ~ 5
    return np.asfortranarray(np.random.default_rng(seed).standard_normal((m, n)))


SHAPES = [(1000, 1000, 100), (1537, 1200, 64), (300, 300, 300), (257, 129, 1), (129, 129, 16), (64, 7, 3),
          (1, 1, 1), (5, 3, 2), (700, 500, 142), (1030, 600, 50), (2000, 1000, 500)]


@pytest.mark.parametrize("m,n,s", SHAPES)
def test_qr_matches_oracle(m, n, s):
    A = matrix(m, n, seed=m + 7 * n + s)
    ws = ff.qr_step(m, n, s)
    assert 1 <= ws <= min(s, n)
    Q, R, info = ff.qr_factor(dev(A), s, sync=True)
    assert info == 0
    Qo, Ro, k, io = oracle.qr_alg3(A, ws)
    assert io == 0 and k == (n - 1) // ws
    Qh, Rh = host(Q), host(R)
    kappa = np.linalg.cond(A)
    dq = np.max(np.abs(Qh - Qo))
    dr = np.max(np.abs(Rh - np.triu(Ro))) / np.max(np.abs(Ro))
    bound = 8 * n * kappa * U
    print(f"m={m} n={n} s={s} (block {ws}): |dQ| = {dq:.2e}, |dR|/|R| = {dr:.2e}, bound {bound:.2e}")
    assert dq <= bound and dr <= bound
    assert np.all(np.tril(Rh, -1) == 0.0)
    assert np.all(np.diag(Rh) > 0)


@pytest.mark.parametrize("m,n,s", [(16, 16, 1), (64, 64, 7), (256, 200, 64), (1024, 1024, 128), (4096, 3000, 142),
                                   (4096, 4096, 100)])
def test_qr_integer_family_bitwise(m, n, s):
    Q0, R0, A = wl.qr_int_family(m, n, seed=m + s)
    Q, R, info = ff.qr_factor(dev(A), s, sync=True)
    assert info == 0
    assert np.array_equal(host(Q), Q0)
    assert np.array_equal(host(R), R0)


def test_qr_fullsize_integer_family_bitwise():
    n = 16384
    Q0, R0, A = wl.qr_int_family_device(n, n, seed=3, device=DEV)
    Q, R, info = ff.qr_factor(A, 128, sync=True)
    assert info == 0
    assert torch.equal(Q, Q0)
    assert torch.equal(R, R0)
    del Q0, R0, A, Q, R
    torch.cuda.empty_cache()


def test_qr_fullsize_benchmark_matrix():
    n, s = 16384, 128
    A = wl.spd_scaled_device(n, seed=0, lam=1.0, device=DEV)    # symmetric: row-major = column-major
    Acm = A.t()
    Q, R, info = ff.qr_factor(Acm, s, sync=True)
    assert info == 0
    ws = ff.qr_step(n, n, s)
    # first three blocks against the oracle
    c = 3 * ws
    Ah = np.asfortranarray(host(Acm[:, :c]))
    Qo, Ro, _, io = oracle.qr_alg3(Ah, ws)
    assert io == 0
    kappa = 5.0      # eigenvalues of G G^T / n lie in [0, 4] (up to finite-n spread), so kappa(A) <= about 5
    dq = float(np.max(np.abs(host(Q[:, :c]) - Qo)))
    dr = float(np.max(np.abs(host(R[:c, :c]) - np.triu(Ro))) / np.max(np.abs(Ro)))
    print(f"first {c} columns: |dQ| = {dq:.2e}, |dR|/|R| = {dr:.2e}")
    assert dq <= 8 * c * kappa * U and dr <= 8 * c * kappa * U
    # whole factorisation: orthogonality and residual (torch binary64 GEMMs)
    QtQ = torch.mm(Q.t(), Q)
    QtQ.diagonal().sub_(1.0)
    orth = float(QtQ.abs().max())
    del QtQ
    res = float((torch.mm(Q, R) - Acm).abs().max() / Acm.abs().max())
    print(f"n={n}: max|Q^T Q - I| = {orth:.2e}, max|QR - A|/max|A| = {res:.2e}")
    assert orth <= 8 * n * kappa * U
    assert res <= 8 * n * U
    assert bool((torch.tril(R, -1) == 0).all())
    assert bool((R.diagonal() > 0).all())
    del A, Acm, Q, R
    torch.cuda.empty_cache()


def test_qr_deterministic():
    A = dev(matrix(1500, 1100, seed=21))
    Q1, R1, i1 = ff.qr_factor(A, 96, sync=True)
    Q2, R2, i2 = ff.qr_factor(A, 96, sync=True)
    assert i1 == i2 == 0
    assert torch.equal(Q1, Q2) and torch.equal(R1, R2)


@pytest.mark.parametrize("col", [0, 5, 130, 299])
def test_qr_zero_column_info(col):
    A = matrix(400, 300, seed=22)
    A[:, col] = 0.0
    _, _, info = ff.qr_factor(dev(A), 64, sync=True)
    _, _, _, io = oracle.qr_alg3(A, ff.qr_step(400, 300, 64))
    assert info == io == col + 1


def test_qr_nan_column_info():
    A = matrix(300, 200, seed=24)
    A[17, 70] = np.nan
    _, _, info = ff.qr_factor(dev(A), 32, sync=True)
    assert info == 71


def test_qr_empty_and_padded_leading_dimensions():
    Q, R, info = ff.qr_factor(ff.colmajor_empty(5, 0, torch.float64, DEV), 4, sync=True)
    assert info == 0 and Q.numel() == 0
    A = matrix(333, 200, seed=25)
    Ad = dev(A, ld=400)
    Qd = ff.colmajor_empty(333, 200, torch.float64, DEV, ld=350)
    Rd = ff.colmajor_empty(200, 200, torch.float64, DEV, ld=256)
    Q, R, info = ff.qr_factor(Ad, 48, Q=Qd, R=Rd, sync=True)
    assert info == 0
    Qo, Ro, _, _ = oracle.qr_alg3(A, ff.qr_step(333, 200, 48))
    assert np.max(np.abs(host(Q) - Qo)) <= 8 * 200 * np.linalg.cond(A) * U


def test_qr_rejects_bad_arguments():
    with pytest.raises(ff.FastFactError):
        ff.qr_factor(dev(np.zeros((10, 20))), 4)  # m < n
    with pytest.raises(ff.FastFactError):
        ff.qr_factor(dev(np.eye(4)), 4, dtype="f32")


def test_qr_tall_matrix_uses_256_row_panel_slices():
    # more rows than 128 per CU: the panel holds 256 rows per workgroup and its
    # block is at most 71 columns wide
    cus = torch.cuda.get_device_properties(DEV).multi_processor_count
    m, n, s = 128 * cus + 1000, 150, 128
    ws = ff.qr_step(m, n, s)
    assert ws <= 71
    A = np.asfortranarray(np.random.default_rng(27).standard_normal((m, n)))
    Q, R, info = ff.qr_factor(dev(A), s, sync=True)
    assert info == 0
    Qo, Ro, _, io = oracle.qr_alg3(A, ws)
    assert io == 0
    kappa = np.linalg.cond(A)
    dq = np.max(np.abs(host(Q) - Qo))
    dr = np.max(np.abs(host(R) - np.triu(Ro))) / np.max(np.abs(Ro))
    print(f"m={m} n={n} (block {ws}): |dQ| = {dq:.2e}, |dR|/|R| = {dr:.2e}")
    assert dq <= 8 * n * kappa * U and dr <= 8 * n * kappa * U


@pytest.mark.parametrize("m,n,s", [(16384, 512, 64), (8192, 1100, 96)])
def test_qr_r_slabs_against_oracle(m, n, s):
    # tall enough that R's tiles are formed over several K chunks beside the
    # panels (stored, then added in K order) and the rest after the last panel
    ws = ff.qr_step(m, n, s)
    A = np.asfortranarray(np.random.default_rng(m + n).standard_normal((m, n)))
    Q, R, info = ff.qr_factor(dev(A), s, sync=True)
    assert info == 0
    Qo, Ro, _, io = oracle.qr_alg3(A, ws)
    assert io == 0
    kappa = np.linalg.cond(A)
    dq = np.max(np.abs(host(Q) - Qo))
    dr = np.max(np.abs(host(R) - np.triu(Ro))) / np.max(np.abs(Ro))
    print(f"m={m} n={n} (block {ws}): |dQ| = {dq:.2e}, |dR|/|R| = {dr:.2e}")
    assert dq <= 8 * n * kappa * U and dr <= 8 * n * kappa * U
    assert bool((torch.tril(R, -1) == 0).all())


def test_qr_r_slabs_with_padded_leading_dimensions():
    # the slab kernel addresses Q, A and R through their own leading dimensions
    m, n, s = 8192, 700, 96
    ws = ff.qr_step(m, n, s)
    A = np.asfortranarray(np.random.default_rng(31).standard_normal((m, n)))
    Ad = dev(A, ld=m + 8)
    Qd = ff.colmajor_empty(m, n, torch.float64, DEV, ld=m + 24)
    Rd = ff.colmajor_empty(n, n, torch.float64, DEV, ld=n + 40)
    Q, R, info = ff.qr_factor(Ad, s, Q=Qd, R=Rd, sync=True)
    assert info == 0
    Qo, Ro, _, io = oracle.qr_alg3(A, ws)
    assert io == 0
    kappa = np.linalg.cond(A)
    assert np.max(np.abs(host(Q) - Qo)) <= 8 * n * kappa * U
    assert np.max(np.abs(host(R) - np.triu(Ro))) / np.max(np.abs(Ro)) <= 8 * n * kappa * U
