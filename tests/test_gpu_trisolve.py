"""GPU parity of the triangular solves (chol_trisolve) against the CPU oracle.

X = L^-T L^-1 B with L the oracle's Cholesky factor, checked against the
oracle's forward + backward substitution.  Sizes cover one block, the blocks
the solving workgroup folds by itself only (n <= 64 * 5), helpers, a ragged
last block, padded leading dimensions and 1..33 right-hand sides (sweeps of at
most 16 columns).  Bounds: relative forward error <= 1e-13 in binary64 and
<= 2e-5 in binary32 (kappa(A) ~ 5, so kappa(L) ~ 2); exact on the integer
family (every intermediate an integer or a dyadic rational of fewer than 53
significant bits; the 64 x 64 block inverses of this family are exact too),
in binary64.
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
TOL = {"f64": 1e-13, "f32": 2e-5}
STORE = {"f64": torch.float64, "f32": torch.float32}


def dev(a, dtype=None, ld=None):
    return ff.to_device(a, DEV, dtype=dtype, ld=ld)


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def run_trisolve(L, B, dtype, ldl=None, ldx=None):
    Ld = dev(L, dtype=STORE[dtype], ld=ldl)
    Xd = dev(B, dtype=STORE[dtype], ld=ldx)
    n = L.shape[0]
    ws = torch.zeros(ff.trisolve_workspace_size(n, dtype), dtype=torch.uint8, device=DEV)
    ff.chol_trisolve(Ld, Xd, dtype=dtype, ws=ws)
    torch.cuda.synchronize()
    err = int(ws[:4].view(torch.int32).item())     # the error word: first int32 of the workspace
    return host(Xd), err


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n", [1, 5, 63, 64, 65, 320, 321, 385, 700, 2000, 4097])
def test_trisolve_sizes(dtype, n):
    A = wl.spd_scaled(n, seed=n)
    Lo, info = oracle.chol(A)
    assert info == 0
    B = wl.rhs(n, 2, seed=n + 1)
    X, err = run_trisolve(Lo, B, dtype)
    assert err == 0
    assert oracle.fwd_x(X, oracle.chol_solve(Lo, B)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("nrhs", [1, 3, 4, 5, 16, 17, 33])
def test_trisolve_rhs_counts(dtype, nrhs):
    n = 1100
    A = wl.spd_scaled(n, seed=31)
    Lo, _ = oracle.chol(A)
    B = wl.rhs(n, nrhs, seed=32)
    X, err = run_trisolve(Lo, B, dtype)
    assert err == 0
    Xo = oracle.chol_solve(Lo, B)
    for c in range(nrhs):
        assert oracle.fwd_x(X[:, c:c + 1], Xo[:, c:c + 1]) <= TOL[dtype], c


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_trisolve_padded_leading_dimensions(dtype):
    n = 777
    A = wl.spd_scaled(n, seed=33)
    Lo, _ = oracle.chol(A)
    B = wl.rhs(n, 6, seed=34)
    X, err = run_trisolve(Lo, B, dtype, ldl=n + 13, ldx=n + 5)
    assert err == 0
    assert oracle.fwd_x(X, oracle.chol_solve(Lo, B)) <= TOL[dtype]


@pytest.mark.parametrize("n", [130, 700, 1500])
def test_trisolve_integer_family_exact(n):
    # binary64 only: the family's 64 x 64 block inverses can need more than the
    # 24 significant bits of binary32
    L0, A = wl.chol_int_family(n, seed=35)
    x0 = np.random.default_rng(36).integers(-1, 2, size=(n, 3)).astype(np.float64)
    B = A @ x0
    X, err = run_trisolve(L0, B, "f64")
    assert err == 0
    assert np.array_equal(X, x0)


def test_trisolve_matches_across_repeats():
    # the sums are taken in a fixed order: repeating the solve gives the same bits
    n = 2500
    A = wl.spd_scaled(n, seed=37)
    Lo, _ = oracle.chol(A)
    B = wl.rhs(n, 5, seed=38)
    X1, e1 = run_trisolve(Lo, B, "f64")
    X2, e2 = run_trisolve(Lo, B, "f64")
    assert e1 == 0 and e2 == 0
    assert np.array_equal(X1, X2)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_trisolve_fullsize(dtype):
    # the benchmark's order, n = 16384: the oracle's substitution on the CPU.  L has
    # diagonal U(1, 2) and strictly lower N(0, 1/n^2) entries, so ||L - diag(L)||_2
    # is about 2 n^-1/2 and kappa(L) is about 2.
    n = 16384
    Lt = torch.tril(torch.randn(n, n, dtype=torch.float64, generator=torch.Generator().manual_seed(39)) / n, -1)
    Lt.diagonal().copy_(1.0 + torch.rand(n, dtype=torch.float64, generator=torch.Generator().manual_seed(40)))
    L = Lt.numpy()
    B = wl.rhs(n, 2, seed=41)
    X, err = run_trisolve(L, B, dtype)
    assert err == 0
    Xo = oracle.chol_solve(L, B)
    assert oracle.fwd_x(X, Xo) <= (1e-12 if dtype == "f64" else 1e-4)
