"""The binary64 residual of the refined solves at the edges of its tile layout.

R = B - A X is formed from tril(A) by 64 x 64 tiles grouped into squares of 4 x 4
tiles, each partial sum stored in a packed per-segment slot and the slots added
in a fixed order.  Sizes below cover one tile and one segment, ragged last
blocks and segments (n = 63, 65, 255, 257, 1030), and right-hand-side counts
below, at and past the 16 columns of one pass.  Binary32 factors with binary64
refinement only reach the oracle's solution when every residual is right, so
each case checks the refined X against the CPU oracle (kappa about 5, bound
1e-12), the library's reported backward error and the same quantity computed
on the host in binary64.
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


def host_backward_error(A, X, B):
    R = B - A @ X
    anorm = np.max(np.sum(np.abs(A), axis=1))
    return float(np.max(np.max(np.abs(R), axis=0) / (anorm * np.max(np.abs(X), axis=0) + np.max(np.abs(B), axis=0))))


@pytest.mark.parametrize("n", [1, 5, 63, 65, 255, 256, 257, 700, 1030])
@pytest.mark.parametrize("nrhs", [1, 3, 17, 33])
def test_refined_solve_across_residual_layout(n, nrhs):
    A = wl.spd_scaled(n, seed=n + 11, lam=1.0)
    B = wl.rhs(n, nrhs, seed=n + 12)
    Lo, oinfo = oracle.chol(A)
    assert oinfo == 0
    Xo = oracle.chol_solve(Lo, B)
    X, _, info = ff.chol_solve(ff.to_device(A, DEV), ff.to_device(B, DEV), 64, dtype="f32", tol=1e-13, max_iter=30)
    Xh = X.cpu().numpy()
    assert info["info"] == 0 and info["converged"] == 1
    fwd = float(np.max(np.abs(Xh - Xo)) / np.max(np.abs(Xo)))
    bwd = host_backward_error(A, Xh, B)
    print(f"n={n} nrhs={nrhs}: {info['iters']} refinements, fwd {fwd:.1e}, bwd {bwd:.1e} "
          f"(library {info['backward_err']:.1e})")
    assert fwd <= 1e-12
    assert bwd <= 1e-14 and info["backward_err"] <= 1e-14


@pytest.mark.parametrize("n,lda", [(257, 300), (700, 768), (1030, 1031)])
def test_refined_solve_with_padded_leading_dimension(n, lda):
    A = wl.spd_scaled(n, seed=n + 21, lam=1.0)
    B = wl.rhs(n, 5, seed=n + 22)
    Lo, _ = oracle.chol(A)
    Xo = oracle.chol_solve(Lo, B)
    X, _, info = ff.chol_solve(ff.to_device(A, DEV, ld=lda), ff.to_device(B, DEV, ld=n + 3), 64, dtype="f32",
                               tol=1e-13, max_iter=30)
    Xh = X.cpu().numpy()
    assert info["info"] == 0 and info["converged"] == 1
    assert float(np.max(np.abs(Xh - Xo)) / np.max(np.abs(Xo))) <= 1e-12
    assert host_backward_error(A, Xh, B) <= 1e-14
