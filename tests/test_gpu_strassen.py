"""GPU parity of the one-level Strassen update (FF_FLAG_STRASSEN1) against the
oracle's definition of the product, through the C ABI.

Strassen's form changes the rounding, not the result.  Error bound used here
(one level; K2 = ceil(K / 2) the length of each half-K product, u = 2^-53,
mx = max|X|, my = max|Y|): each of the seven products has operands that are sums
of two entries (|.| <= 2 mx, 2 my), so its computed value is within
(K2 + 2) u * 4 K2 mx my of the exact product of the exact sums; a quadrant adds at
most four products with three roundings and then subtracts from C:
    |computed - exact| <= (16 K2 (K2 + 5) + K) u mx my + 2 u |C|   elementwise.
Diagonal super-tiles of the Cholesky update take the classical products and
satisfy this bound too.  On the integer families every sum and product is a small
integer, so results are bit-exact.
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
U = 2.0 ** -53


def dev(a, dtype=None, ld=None):
    return ff.to_device(a, DEV, dtype=dtype, ld=ld)


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def strassen_bound(K, C, mx, my):
    K2 = (K + 1) // 2
    return (16.0 * K2 * (K2 + 5) + K) * U * mx * my + 2 * U * np.abs(C)


SHAPES = [(1, 1), (5, 3), (63, 2), (64, 16), (127, 16), (128, 16), (129, 17), (300, 27), (513, 118),
          (260, 256), (1100, 64), (257, 512), (700, 1)]


@pytest.mark.parametrize("m,w", SHAPES)
def test_strassen_syrk_f64(m, w):
    rng = np.random.default_rng(31 * m + w)
    C = rng.standard_normal((m, m))
    P = rng.standard_normal((m, w))
    ld = m + 3
    Cd = dev(C, ld=ld)
    ff.update_syrk(Cd, dev(P, ld=ld + 1), dtype="f64", strassen=True)
    got = host(Cd)
    ref = oracle.syrk_update(C, P)
    mp = np.abs(P).max()
    bound = strassen_bound(w, C, mp, mp)
    assert np.all(np.abs(np.tril(got) - np.tril(ref)) <= np.tril(bound))
    assert np.array_equal(np.triu(got, 1), np.triu(C, 1))


@pytest.mark.parametrize("m,w", [(129, 17), (300, 27), (700, 168), (257, 512), (640, 255)])
def test_strassen_syrk_f64_integer_exact(m, w):
    rng = np.random.default_rng(m + 3 * w)
    C = rng.integers(-100, 100, size=(m, m)).astype(np.float64)
    P = rng.integers(-2, 3, size=(m, w)).astype(np.float64)
    Cd = dev(C)
    ff.update_syrk(Cd, dev(P), dtype="f64", strassen=True)
    got = host(Cd)
    assert np.array_equal(np.tril(got), np.tril(oracle.syrk_update(C, P)))
    assert np.array_equal(np.triu(got, 1), np.triu(C, 1))


@pytest.mark.parametrize("m,w", [(1, 1), (65, 3), (129, 17), (300, 27), (700, 168), (513, 256), (384, 511)])
def test_strassen_gemm_f64(m, w):
    rng = np.random.default_rng(13 * m + w)
    C = rng.standard_normal((m, m))
    X = rng.standard_normal((m, w))
    Y = rng.standard_normal((w, m))
    Cd = dev(C, ld=m + 1)
    ff.update_gemm(Cd, dev(X, ld=m + 2), dev(Y, ld=w + 5), dtype="f64", strassen=True)
    got = host(Cd)
    ref = oracle.gemm_update(C, X, Y)
    assert np.all(np.abs(got - ref) <= strassen_bound(w, C, np.abs(X).max(), np.abs(Y).max()))
    Ci = rng.integers(-50, 50, size=(m, m)).astype(np.float64)
    Xi = rng.integers(-2, 3, size=(m, w)).astype(np.float64)
    Yi = rng.integers(-2, 3, size=(w, m)).astype(np.float64)
    Cd = dev(Ci)
    ff.update_gemm(Cd, dev(Xi), dev(Yi), dtype="f64", strassen=True)
    assert np.array_equal(host(Cd), oracle.gemm_update(Ci, Xi, Yi))


def test_strassen_differs_from_classical_only_by_rounding():
    # same inputs through both forms: equal within the bound, and not bitwise equal
    # in general (the seven products are really used)
    rng = np.random.default_rng(2)
    m, w = 520, 200
    C = rng.standard_normal((m, m))
    P = rng.standard_normal((m, w))
    Pd = dev(P)
    C1, C2 = dev(C), dev(C)
    ff.update_syrk(C1, Pd, dtype="f64")
    ff.update_syrk(C2, Pd, dtype="f64", strassen=True)
    a, b = np.tril(host(C1)), np.tril(host(C2))
    mp = np.abs(P).max()
    assert np.all(np.abs(a - b) <= 2 * np.tril(strassen_bound(w, C, mp, mp)))
    assert not np.array_equal(a, b)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_strassen_other_dtypes_unsupported(dtype):
    C = dev(np.eye(8), dtype=torch.float32)
    P = dev(np.ones((8, 2)), dtype=torch.float32)
    with pytest.raises(ff.FastFactError):
        ff.update_syrk(C, P, dtype=dtype, strassen=True)


@pytest.mark.parametrize("n,s", [(3, 2), (200, 27), (512, 28), (1000, 118), (777, 168), (1300, 256)])
@pytest.mark.parametrize("no_lookahead", [False, True])
def test_strassen_chol_integer_family_bitwise(n, s, no_lookahead):
    L0, A = wl.chol_int_family(n, seed=n + 2 * s)
    Ad = dev(A, ld=n + 5)
    assert ff.chol_factor(Ad, s, dtype="f64", strassen=True, no_lookahead=no_lookahead, sync=True) == 0
    assert np.array_equal(np.tril(host(Ad)), L0)


@pytest.mark.parametrize("s", [64, 168, 256])
def test_strassen_chol_scaled_family(s):
    n = 2048
    A = wl.spd_scaled(n, seed=41)
    Ad = dev(A)
    assert ff.chol_factor(Ad, s, dtype="f64", strassen=True, sync=True) == 0
    L = np.tril(host(Ad))
    Lo, _ = oracle.chol(A)
    assert oracle.rel_lower(L, Lo) <= 1e-11
    assert oracle.bwd_chol(A, L) <= 1e-13


@pytest.mark.parametrize("n,s", [(13, 4), (300, 27), (513, 168), (1100, 256)])
def test_strassen_lu_integer_family_bitwise(n, s):
    L0, U0, A = wl.lu_int_family(n, seed=5 * n + s)
    Ad = dev(A, ld=n + 2)
    assert ff.lu_nopiv_factor(Ad, s, dtype="f64", strassen=True, sync=True) == 0
    LU = host(Ad)
    assert np.array_equal(np.tril(LU, -1) + np.eye(n), L0)
    assert np.array_equal(np.triu(LU), U0)


def test_strassen_lu_diag_dominant():
    n, s = 1536, 168
    A = wl.diag_dominant(n, seed=9)
    Ad = dev(A)
    assert ff.lu_nopiv_factor(Ad, s, dtype="f64", strassen=True, sync=True) == 0
    LU = host(Ad)
    LUo, _ = oracle.lu(A)
    Lg, Lo = np.tril(LU, -1), np.tril(LUo, -1)
    Ug, Uo = np.triu(LU), np.triu(LUo)
    assert np.linalg.norm(Lg - Lo) / np.linalg.norm(Lo + np.eye(n)) <= 1e-11
    assert np.linalg.norm(Ug - Uo) / np.linalg.norm(Uo) <= 1e-11
    assert oracle.bwd_lu(A, LU) <= 1e-13


def test_strassen_update_skipped_when_info_set():
    # the factorisation's info word stops the update kernels: a non-SPD leading
    # block leaves the trailing matrix as the failed step left it, in both forms
    L0, A = wl.chol_int_family(600, seed=77)
    A[10, 10] -= L0[10, 10] ** 2 + 1.0
    A1, A2 = dev(A), dev(A)
    i1 = ff.chol_factor(A1, 64, dtype="f64", sync=True, no_lookahead=True)
    i2 = ff.chol_factor(A2, 64, dtype="f64", strassen=True, sync=True, no_lookahead=True)
    assert i1 == i2 == 11
    assert np.array_equal(host(A1), host(A2))


# Two Strassen levels (FF_FLAG_STRASSEN2): a matrix-level level over the
# one-level kernel on trailing products of m >= 2048 rows.  On the integer family
# every operand sum, product and accumulation stays a small integer, so the
# factors must be the generating ones bit for bit; odd n and odd steps exercise the
# classical remainders of the matrix-level split.
@pytest.mark.parametrize("n,s,no_lookahead", [(4096, 256, False), (4097, 257, False), (4400, 384, True),
                                              (2600, 129, False)])
def test_strassen2_lu_integer_family_bitwise(n, s, no_lookahead):
    L0, U0, A = wl.lu_int_family(n, seed=3 * n + s)
    Ad = dev(A, ld=n + 3)
    assert ff.lu_nopiv_factor(Ad, s, dtype="f64", strassen=2, no_lookahead=no_lookahead, sync=True) == 0
    LU = host(Ad)
    assert np.array_equal(np.tril(LU, -1) + np.eye(n), L0)
    assert np.array_equal(np.triu(LU), U0)


def test_strassen2_lu_diag_dominant_against_oracle():
    # two levels: operand sums of up to four entries and Strassen's constant grown
    # by about 12 per level (Higham, Accuracy and Stability, Sec. 23.2.2); the
    # factors of this well-conditioned matrix stay within 1e-10 of the oracle's
    n, s = 3000, 384
    A = wl.diag_dominant(n, seed=19)
    Ad = dev(A)
    assert ff.lu_nopiv_factor(Ad, s, dtype="f64", strassen=2, sync=True) == 0
    LU = host(Ad)
    LUo, _ = oracle.lu(A)
    Lg, Lo = np.tril(LU, -1), np.tril(LUo, -1)
    Ug, Uo = np.triu(LU), np.triu(LUo)
    el = np.linalg.norm(Lg - Lo) / np.linalg.norm(Lo + np.eye(n))
    eu = np.linalg.norm(Ug - Uo) / np.linalg.norm(Uo)
    print(f"two-level Strassen LU n={n} s={s}: rel_L {el:.2e} rel_U {eu:.2e} bwd {oracle.bwd_lu(A, LU):.2e}")
    assert el <= 1e-10 and eu <= 1e-10
    assert oracle.bwd_lu(A, LU) <= 1e-12


def test_strassen2_lu_fullsize_integer_family_bitwise():
    n, s = 16384, 768
    L0, U0, A = wl.lu_int_family_device(n, seed=23, device=DEV)
    Acm = A.t().contiguous().t()
    assert ff.lu_nopiv_factor(Acm, s, dtype="f64", strassen=2, sync=True) == 0
    assert torch.equal(torch.tril(Acm, -1) + torch.eye(n, dtype=torch.float64, device=DEV), L0)
    assert torch.equal(torch.triu(Acm), U0)
    del L0, U0, A, Acm
    torch.cuda.empty_cache()
