"""GMRES-based iterative refinement (FF_FLAG_GMRES_IR): each refinement step
solves its correction equation by GMRES in binary64, preconditioned by the
low-precision factor, rather than by one pair of triangular solves.  Results
are checked against the CPU oracle's solution on the configuration's
matrices A = G G^T / n + lambda I (lambda = 1e-3: kappa ~ 4e3; 1e-6: kappa ~ 4e6).

Accuracy criterion as for the classical refinement: backward error <= 1e-12
for every result, and forward error against the oracle <= 1e-12 wherever two
independent binary64 solvers agree that closely.
"""
import numpy as np
import pytest

import oracle
from paper_1812_02056_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
scipy_linalg = pytest.importorskip("scipy.linalg")

import paper_1812_02056_amd as ff  # noqa: E402

DEV = torch.device("cuda:0")
N, S = 2000, 256
DT = {"f64": 0, "f32": 1, "bf16": 2}


def dev(a):
    return ff.to_device(a, DEV)


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module", params=[1e-3, 1e-6], ids=["lam1e-3", "lam1e-6"])
def system(request):
    lam = request.param
    A = wl.spd_scaled(N, seed=71, lam=lam)
    B = wl.rhs(N, 2, seed=72)
    Lo, info = oracle.chol(A)
    assert info == 0
    Xo = oracle.chol_solve(Lo, B)
    Xl = scipy_linalg.cho_solve(scipy_linalg.cho_factor(A, lower=True), B)
    return lam, A, B, Xo, oracle.fwd_x(Xl, Xo)


def check(A, B, Xo, d64, X, info, label):
    Xh = host(X)
    fx, bx = oracle.fwd_x(Xh, Xo), oracle.bwd_x(A, Xh, B)
    print(f"{label}: used={info['dtype_used']} iters={info['iters']} krylov={info['krylov_iters']} "
          f"conv={info['converged']} fwd_x={fx:.2e} bwd_x={bx:.2e} (binary64 solvers differ by {d64:.1e})")
    assert info["info"] == 0
    assert bx <= 1e-12
    if d64 <= 1e-12:
        assert fx <= 1e-12


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_gmres_ir_accuracy(system, dtype):
    lam, A, B, Xo, d64 = system
    X, _, info = ff.chol_solve(dev(A), dev(B), S, dtype=dtype, tol=1e-12, max_iter=20, gmres=True,
                               escalate=True)
    check(A, B, Xo, d64, X, info, f"lam={lam:g} {dtype}")
    assert info["krylov_iters"] > 0
    if dtype == "bf16" and lam == 1e-6:
        # the bfloat16-operand factor breaks down there; binary32 + GMRES serves
        assert info["escalated_to"] in (DT["f32"], DT["f64"])


def test_gmres_ir_fewer_outer_steps_than_classical(system):
    """At kappa ~ 4e3 classical refinement with the bfloat16 factor contracts
    slowly; GMRES-IR reaches the same accuracy in a few outer steps."""
    lam, A, B, Xo, d64 = system
    if lam != 1e-3:
        pytest.skip("the bfloat16 factor exists only at lambda = 1e-3")
    Xc, _, ic = ff.chol_solve(dev(A), dev(B), S, dtype="bf16", tol=1e-12, max_iter=100)
    Xg, _, ig = ff.chol_solve(dev(A), dev(B), S, dtype="bf16", tol=1e-12, max_iter=20, gmres=True)
    print(f"classical: iters={ic['iters']} conv={ic['converged']}  gmres: outer={ig['iters']} "
          f"krylov={ig['krylov_iters']} conv={ig['converged']}")
    check(A, B, Xo, d64, Xg, ig, "gmres bf16")
    assert ig["escalated_to"] == -1 and ig["dtype_used"] == DT["bf16"]
    assert ig["iters"] <= 4
    assert ig["iters"] < ic["iters"]


def test_gmres_ir_binary64_factor_matches_classical(system):
    """With a binary64 factor both refinements reach the oracle's solution."""
    lam, A, B, Xo, d64 = system
    X, _, info = ff.chol_solve(dev(A), dev(B), S, dtype="f64", tol=1e-14, max_iter=5, gmres=True)
    check(A, B, Xo, d64, X, info, f"lam={lam:g} f64")
    assert info["iters"] <= 3


def test_gmres_ir_zero_rhs_column():
    """A zero right-hand side gives x = 0 exactly (GMRES starts from a zero
    residual and takes no step), beside a nonzero column."""
    A = wl.spd_scaled(700, seed=73, lam=1e-3)
    B = wl.rhs(700, 2, seed=74)
    B[:, 1] = 0.0
    X, _, info = ff.chol_solve(dev(A), dev(B), 128, dtype="f32", tol=1e-12, max_iter=20, gmres=True)
    Xh = host(X)
    assert np.all(Xh[:, 1] == 0.0)
    Lo, _ = oracle.chol(A)
    assert oracle.fwd_x(Xh[:, :1], oracle.chol_solve(Lo, B[:, :1])) <= 1e-12
    assert info["info"] == 0


@pytest.mark.parametrize("n,nrhs", [(65, 3), (257, 17), (1030, 16)])
def test_gmres_ir_ragged_sizes(n, nrhs):
    """Ragged sizes and right-hand-side counts past one 16-column pass: the
    Krylov matrix products run through the residual's tile layout."""
    A = wl.spd_scaled(n, seed=n + 75, lam=1e-3)
    B = wl.rhs(n, nrhs, seed=n + 76)
    Lo, info_o = oracle.chol(A)
    assert info_o == 0
    Xo = oracle.chol_solve(Lo, B)
    X, _, info = ff.chol_solve(dev(A), dev(B), 64, dtype="f32", tol=1e-12, max_iter=20, gmres=True)
    Xh = host(X)
    assert info["info"] == 0 and info["converged"] == 1 and info["krylov_iters"] > 0
    assert oracle.bwd_x(A, Xh, B) <= 1e-12
    # kappa ~ 4e3: a backward error of 1e-12 bounds the forward error by about
    # kappa * 1e-12 = 4e-9; binary64 itself lands near kappa * u ~ 1e-12
    assert oracle.fwd_x(Xh, Xo) <= 1e-10
