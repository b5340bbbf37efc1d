"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Tolerances (binary64 path): ||tril(L - L_oracle)||_F / ||tril(L)||_F <= 1e-11 for
kappa <= 1e3, backward error ||A - L L^T||_F / ||A||_F <= 1e-13, and bit-exact
equality on the integer families, where every intermediate of any evaluation
order is an exactly representable integer.

Update-kernel bound (binary32 / bfloat16 operand paths): each entry of C - P P^T is
a sum of w products accumulated in binary32, so
|gpu - exact| <= (w + 2) * 2^-24 * (|C| + sum_k |P_ik P_jk|) elementwise, where
"exact" is computed by the oracle in binary64 on the operands as rounded by the
path (binary32 storage, and bfloat16 rounding for the bf16 variant).
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


def dev(a, dtype=None, ld=None):
    return ff.to_device(a, DEV, dtype=dtype, ld=ld)


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


# --------------------------------------------------------------------------- update kernel

UPDATE_SHAPES = [(1, 1), (5, 3), (16, 4), (127, 16), (128, 16), (129, 17), (300, 27), (513, 118),
                 (700, 168), (260, 256), (1100, 64), (257, 512)]


@pytest.mark.parametrize("m,w", UPDATE_SHAPES)
def test_update_syrk_f64(m, w):
    rng = np.random.default_rng(m * 1000 + w)
    C = rng.standard_normal((m, m))
    P = rng.standard_normal((m, w))
    ld = m + 3
    Cd = dev(C, ld=ld)
    ff.update_syrk(Cd, dev(P, ld=ld), dtype="f64")
    got = host(Cd)
    ref = oracle.syrk_update(C, P)
    scale = np.abs(C) + np.abs(P) @ np.abs(P).T
    assert np.all(np.abs(np.tril(got) - np.tril(ref)) <= (w + 2) * 2.0 ** -53 * np.tril(scale) + 1e-300)
    assert np.array_equal(np.triu(got, 1), np.triu(C, 1))


@pytest.mark.parametrize("m,w", [(129, 17), (300, 27), (700, 168), (257, 512)])
def test_update_syrk_f64_integer_exact(m, w):
    rng = np.random.default_rng(m + w)
    C = rng.integers(-100, 100, size=(m, m)).astype(np.float64)
    P = rng.integers(-2, 3, size=(m, w)).astype(np.float64)
    Cd = dev(C)
    ff.update_syrk(Cd, dev(P), dtype="f64")
    got = host(Cd)
    assert np.array_equal(np.tril(got), np.tril(oracle.syrk_update(C, P)))
    assert np.array_equal(np.triu(got, 1), np.triu(C, 1))


@pytest.mark.parametrize("m,w", [(1, 1), (129, 17), (300, 27), (700, 168), (513, 256)])
def test_update_gemm_f64(m, w):
    rng = np.random.default_rng(7 * m + w)
    C = rng.standard_normal((m, m))
    X = rng.standard_normal((m, w))
    Y = rng.standard_normal((w, m))
    Cd = dev(C, ld=m + 1)
    ff.update_gemm(Cd, dev(X, ld=m + 2), dev(Y, ld=w + 5), dtype="f64")
    got = host(Cd)
    ref = oracle.gemm_update(C, X, Y)
    scale = np.abs(C) + np.abs(X) @ np.abs(Y)
    assert np.all(np.abs(got - ref) <= (w + 2) * 2.0 ** -53 * scale)
    Ci = rng.integers(-50, 50, size=(m, m)).astype(np.float64)
    Xi = rng.integers(-2, 3, size=(m, w)).astype(np.float64)
    Yi = rng.integers(-2, 3, size=(w, m)).astype(np.float64)
    Cd = dev(Ci)
    ff.update_gemm(Cd, dev(Xi), dev(Yi), dtype="f64")
    assert np.array_equal(host(Cd), oracle.gemm_update(Ci, Xi, Yi))


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("m,w", [(5, 3), (129, 17), (300, 27), (700, 168), (260, 256)])
def test_update_syrk_low_precision(dtype, m, w):
    rng = np.random.default_rng(11 * m + w)
    C = oracle.round_f32(rng.standard_normal((m, m)))
    P = oracle.round_f32(rng.standard_normal((m, w)))
    Cd = dev(C, dtype=torch.float32)
    ff.update_syrk(Cd, dev(P, dtype=torch.float32), dtype=dtype)
    got = host(Cd)
    Pr = oracle.round_bf16(P) if dtype == "bf16" else P
    ref = oracle.syrk_update(C, Pr)
    scale = np.abs(C) + np.abs(Pr) @ np.abs(Pr).T
    err = np.abs(np.tril(got) - np.tril(ref))
    assert np.all(err <= (w + 2) * 2.0 ** -24 * np.tril(scale))
    assert np.array_equal(np.triu(got, 1), np.triu(C, 1))


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_update_syrk_low_precision_integer_exact(dtype):
    rng = np.random.default_rng(5)
    m, w = 333, 118
    C = rng.integers(-100, 100, size=(m, m)).astype(np.float64)
    P = rng.integers(-1, 3, size=(m, w)).astype(np.float64)      # {-1,0,1,2}: exact in bfloat16
    Cd = dev(C, dtype=torch.float32)
    ff.update_syrk(Cd, dev(P, dtype=torch.float32), dtype=dtype)
    assert np.array_equal(np.tril(host(Cd)), np.tril(oracle.syrk_update(C, P)))


# --------------------------------------------------------------------------- Cholesky

@pytest.mark.parametrize("n,s", [(1, 1), (2, 1), (3, 2), (5, 5), (31, 4), (64, 16), (200, 27), (200, 200),
                                 (512, 27), (512, 28), (1000, 64), (1000, 118), (777, 168), (600, 600),
                                 (1100, 1000)])
def test_chol_f64_integer_family_bitwise(n, s):
    L0, A = wl.chol_int_family(n, seed=n + s)
    Ad = dev(A, ld=n + 5)
    info = ff.chol_factor(Ad, s, dtype="f64", sync=True)
    assert info == 0
    assert np.array_equal(np.tril(host(Ad)), L0)


@pytest.mark.parametrize("s", [27, 28])
def test_chol_f64_config_small(s):
    """A = G G^T + 512 I, n = 512 (kappa ~ 5)."""
    A = wl.spd_shifted(512, seed=0)
    Ad = dev(A)
    assert ff.chol_factor(Ad, s, dtype="f64", sync=True) == 0
    L = np.tril(host(Ad))
    Lo, _ = oracle.chol(A)
    assert oracle.rel_lower(L, Lo) <= 1e-11
    assert oracle.bwd_chol(A, L) <= 1e-13
    # the strict upper triangle is never written
    assert np.array_equal(np.triu(host(Ad), 1), np.triu(A, 1))


@pytest.mark.parametrize("s", [64, 118, 169, 256, 512])
def test_chol_f64_scaled_family_n2048(s):
    A = wl.spd_scaled(2048, seed=1)
    Ad = dev(A, ld=2048 + 8)
    assert ff.chol_factor(Ad, s, dtype="f64", sync=True) == 0
    L = np.tril(host(Ad))
    Lo, _ = oracle.chol(A)
    assert oracle.rel_lower(L, Lo) <= 1e-11
    assert oracle.bwd_chol(A, L) <= 1e-13


def test_chol_f64_known_factor():
    L0, A = wl.chol_float_family(1024, seed=2, scaled=True)
    Ad = dev(A)
    assert ff.chol_factor(Ad, 118, dtype="f64", sync=True) == 0
    assert oracle.rel_lower(np.tril(host(Ad)), L0) <= 1e-12


@pytest.mark.parametrize("k", [0, 5, 63, 64, 130, 299])
def test_chol_info_on_non_spd(k):
    L0, A = wl.chol_int_family(300, seed=3)
    A[k, k] -= L0[k, k] ** 2 + 1.0
    Ad = dev(A)
    info = ff.chol_factor(Ad, 64, dtype="f64", sync=True)
    assert info == k + 1
    # columns of the blocks before the failing one are final
    kb = (k // 64) * 64
    assert np.array_equal(np.tril(host(Ad))[:, :kb], L0[:, :kb])


def test_chol_info_on_nan():
    _, A = wl.chol_int_family(100, seed=4)
    A[40, 40] = np.nan
    assert ff.chol_factor(dev(A), 16, dtype="f64", sync=True) == 41


def test_chol_n_zero_and_tiny():
    Ad = torch.empty((1, 1), dtype=torch.float64, device=DEV)
    assert ff.chol_factor(Ad[:0, :0], 4, dtype="f64", sync=True) == 0
    A = np.array([[4.0]])
    Ad = dev(A)
    assert ff.chol_factor(Ad, 4, dtype="f64", sync=True) == 0
    assert host(Ad)[0, 0] == 2.0


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("n,s", [(200, 27), (700, 168), (600, 600)])
def test_chol_low_precision_integer_family_bitwise(dtype, n, s):
    L0, A = wl.chol_int_family(n, seed=2 * n + s)
    Ad = dev(A, dtype=torch.float32)
    assert ff.chol_factor(Ad, s, dtype=dtype, sync=True) == 0
    assert np.array_equal(np.tril(host(Ad)), L0)


@pytest.mark.parametrize("dtype,bound", [("f32", 1e-5), ("bf16", 1e-2)])
def test_chol_low_precision_error_stated(dtype, bound):
    A = wl.spd_scaled(1024, seed=5)
    Ad = dev(A, dtype=torch.float32)
    assert ff.chol_factor(Ad, 118, dtype=dtype, sync=True) == 0
    Lo, _ = oracle.chol(A)
    rel = oracle.rel_lower(np.tril(host(Ad)), Lo)
    print(f"{dtype} factor rel_L vs binary64 oracle: {rel:.3e}")
    assert rel <= bound


# --------------------------------------------------------------------------- LU

@pytest.mark.parametrize("n,s", [(1, 1), (3, 1), (13, 4), (64, 16), (300, 27), (513, 168), (700, 700)])
def test_lu_f64_integer_family_bitwise(n, s):
    L0, U0, A = wl.lu_int_family(n, seed=n * 3 + s)
    Ad = dev(A, ld=n + 2)
    assert ff.lu_nopiv_factor(Ad, s, dtype="f64", sync=True) == 0
    LU = host(Ad)
    assert np.array_equal(np.tril(LU, -1) + np.eye(n), L0)
    assert np.array_equal(np.triu(LU), U0)


@pytest.mark.parametrize("s", [64, 168, 256])
def test_lu_f64_diag_dominant(s):
    A = wl.diag_dominant(1536, seed=6)
    Ad = dev(A)
    assert ff.lu_nopiv_factor(Ad, s, dtype="f64", sync=True) == 0
    LU = host(Ad)
    LUo, _ = oracle.lu(A)
    Lg, Lo = np.tril(LU, -1), np.tril(LUo, -1)
    Ug, Uo = np.triu(LU), np.triu(LUo)
    assert np.linalg.norm(Lg - Lo) / np.linalg.norm(Lo + np.eye(1536)) <= 1e-11
    assert np.linalg.norm(Ug - Uo) / np.linalg.norm(Uo) <= 1e-11
    assert oracle.bwd_lu(A, LU) <= 1e-13


# Block widths: with s > 192 the first block and the blocks of the last 6144
# columns are 192 wide unless FF_FLAG_FIXED_STEP keeps every block s wide.  The
# factor is unique, so both schedules must reproduce the integer family exactly
# and the oracle within the binary64 tolerance.

@pytest.mark.parametrize("n,s", [(900, 320), (1300, 256), (2000, 384), (1500, 512)])
@pytest.mark.parametrize("fixed_step", [False, True])
@pytest.mark.parametrize("no_lookahead", [False, True])
def test_chol_block_widths_integer_family_bitwise(n, s, fixed_step, no_lookahead):
    L0, A = wl.chol_int_family(n, seed=3 * n + s)
    Ad = dev(A, ld=n + 3)
    assert ff.chol_factor(Ad, s, dtype="f64", fixed_step=fixed_step, no_lookahead=no_lookahead, sync=True) == 0
    assert np.array_equal(np.tril(host(Ad)), L0)


@pytest.mark.parametrize("s", [256, 384])
def test_chol_block_widths_scaled_family(s):
    n = 2048
    A = wl.spd_scaled(n, seed=s)
    Lo, _ = oracle.chol(A)
    out = []
    for fixed in (False, True):
        Ad = dev(A)
        assert ff.chol_factor(Ad, s, dtype="f64", fixed_step=fixed, sync=True) == 0
        L = np.tril(host(Ad))
        assert oracle.rel_lower(L, Lo) <= 1e-11
        assert oracle.bwd_chol(A, L) <= 1e-13
        out.append(L)
    # 192-wide blocks instead of s-wide ones change the rounding, not the factor
    assert not np.array_equal(out[0], out[1])


@pytest.mark.parametrize("n,s", [(2000, 384), (1300, 320)])
def test_chol_fixed_step_lookahead_matches_in_order_bitwise(n, s):
    A = wl.spd_scaled(n, seed=n + s)
    A1, A2 = dev(A), dev(A)
    assert ff.chol_factor(A1, s, fixed_step=True, sync=True) == 0
    assert ff.chol_factor(A2, s, fixed_step=True, no_lookahead=True, sync=True) == 0
    assert np.array_equal(host(A1), host(A2))


# LU block widths: with s > 128 the first block and the blocks of the last 4096
# columns are 128 wide unless FF_FLAG_FIXED_STEP keeps every block s wide.

@pytest.mark.parametrize("n,s", [(700, 256), (1300, 384), (2100, 768)])
@pytest.mark.parametrize("fixed_step", [False, True])
@pytest.mark.parametrize("no_lookahead", [False, True])
def test_lu_block_widths_integer_family_bitwise(n, s, fixed_step, no_lookahead):
    L0, U0, A = wl.lu_int_family(n, seed=7 * n + s)
    Ad = dev(A, ld=n + 1)
    assert ff.lu_nopiv_factor(Ad, s, fixed_step=fixed_step, no_lookahead=no_lookahead, sync=True) == 0
    LU = host(Ad)
    assert np.array_equal(np.tril(LU, -1) + np.eye(n), L0)
    assert np.array_equal(np.triu(LU), U0)


@pytest.mark.parametrize("fixed_step", [False, True])
def test_lu_block_widths_diag_dominant(fixed_step):
    n, s = 1536, 384
    A = wl.diag_dominant(n, seed=13)
    Ad = dev(A)
    assert ff.lu_nopiv_factor(Ad, s, fixed_step=fixed_step, sync=True) == 0
    LU = host(Ad)
    LUo, _ = oracle.lu(A)
    Lg, Lo = np.tril(LU, -1), np.tril(LUo, -1)
    Ug, Uo = np.triu(LU), np.triu(LUo)
    assert np.linalg.norm(Lg - Lo) / np.linalg.norm(Lo + np.eye(n)) <= 1e-11
    assert np.linalg.norm(Ug - Uo) / np.linalg.norm(Uo) <= 1e-11
    assert oracle.bwd_lu(A, LU) <= 1e-13


@pytest.mark.parametrize("n,s", [(1000, 64), (1300, 168), (2000, 256), (2100, 768)])
def test_lu_lookahead_matches_in_order_bitwise(n, s):
    # the lookahead schedule splits each update into strips and a remainder (and a
    # tail on the other stream); every entry sees the same products in the same order
    A = wl.diag_dominant(n, seed=n + s)
    A1, A2 = dev(A), dev(A)
    assert ff.lu_nopiv_factor(A1, s, sync=True) == 0
    assert ff.lu_nopiv_factor(A2, s, no_lookahead=True, sync=True) == 0
    assert np.array_equal(host(A1), host(A2))


def test_lu_info_on_zero_pivot():
    L0, U0, _ = wl.lu_int_family(200, seed=8)
    U0[70, 70] = 0.0
    Ad = dev(L0 @ U0)
    assert ff.lu_nopiv_factor(Ad, 32, dtype="f64", sync=True) == 71


# --------------------------------------------------------------------------- solves

@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_trisolve(dtype):
    n, nrhs = 700, 3
    A = wl.spd_scaled(n, seed=9)
    Lo, _ = oracle.chol(A)
    B = wl.rhs(n, nrhs, seed=10)
    st = torch.float64 if dtype == "f64" else torch.float32
    Xd = dev(B, dtype=st)
    ff.chol_trisolve(dev(Lo, dtype=st), Xd, dtype=dtype)
    torch.cuda.synchronize()
    Xo = oracle.chol_solve(Lo, B)
    tol = 1e-13 if dtype == "f64" else 1e-5
    assert oracle.fwd_x(host(Xd), Xo) <= tol


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("nrhs", [1, 16, 19])
def test_chol_solve_refined(dtype, nrhs):
    n = 1000
    A = wl.spd_scaled(n, seed=11, lam=1.0)
    B = wl.rhs(n, nrhs, seed=12)
    X, _, info = ff.chol_solve(dev(A), dev(B), 118, dtype=dtype, tol=1e-13, max_iter=50)
    Lo, _ = oracle.chol(A)
    Xo = oracle.chol_solve(Lo, B)
    fx = oracle.fwd_x(host(X), Xo)
    bx = oracle.bwd_x(A, host(X), B)
    print(f"{dtype} nrhs={nrhs}: iters={info['iters']} fwd_x={fx:.2e} bwd_x={bx:.2e} lib_bwd={info['backward_err']:.2e}")
    assert info["info"] == 0
    assert fx <= 1e-12
    assert bx <= 1e-15
    # the library's own certificate (its residual is itself computed in binary64,
    # so at this level the two values only agree in magnitude)
    assert info["backward_err"] <= 1e-15


def test_chol_solve_integer_exact_no_refinement():
    n = 300
    L0, A = wl.chol_int_family(n, seed=13)
    x0 = np.random.default_rng(13).integers(-1, 2, size=(n, 2)).astype(np.float64)
    X, W, info = ff.chol_solve(dev(A), dev(A @ x0), 64, dtype="f64", max_iter=3)
    assert info["info"] == 0
    assert np.array_equal(np.tril(host(W)), L0)
    assert oracle.fwd_x(host(X), x0) <= 1e-13


def test_chol_solve_reports_non_spd():
    L0, A = wl.chol_int_family(128, seed=14)
    A[77, 77] -= L0[77, 77] ** 2 + 1.0
    _, _, info = ff.chol_solve(dev(A), dev(wl.rhs(128, 1, 1)), 32, dtype="f32")
    assert info["info"] == 78


def test_chol_solve_resident_factor_reuse():
    n = 512
    A = wl.spd_scaled(n, seed=15)
    B1, B2 = wl.rhs(n, 2, seed=16), wl.rhs(n, 3, seed=17)
    Ad = dev(A)
    X1, W, i1 = ff.chol_solve(Ad, dev(B1), 64, dtype="f32")
    X2, _, i2 = ff.chol_solve(Ad, dev(B2), 64, dtype="f32", W=W, w_is_factored=True)
    Lo, _ = oracle.chol(A)
    assert oracle.fwd_x(host(X2), oracle.chol_solve(Lo, B2)) <= 1e-12
    assert i2["converged"] == 1


# --------------------------------------------------------------------------- schedule invariance

@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("n,s", [(1000, 64), (1000, 200), (1300, 256)])
def test_chol_lookahead_matches_in_order_bitwise(dtype, n, s):
    """Lookahead only reorders independent work and splits the update into two
    launches; every element sees the same operations, so the factor is bitwise
    the same as with the strictly ordered schedule."""
    A = wl.spd_scaled(n, seed=21)
    st = torch.float64 if dtype == "f64" else torch.float32
    A1, A2 = dev(A, dtype=st), dev(A, dtype=st)
    assert ff.chol_factor(A1, s, dtype=dtype, sync=True) == 0
    assert ff.chol_factor(A2, s, dtype=dtype, no_lookahead=True, sync=True) == 0
    assert torch.equal(A1, A2)


def test_chol_deterministic_repeat():
    A = wl.spd_scaled(1500, seed=22)
    outs = []
    for _ in range(2):
        Ad = dev(A)
        assert ff.chol_factor(Ad, 168, dtype="f64", sync=True) == 0
        outs.append(Ad)
    assert torch.equal(outs[0], outs[1])
