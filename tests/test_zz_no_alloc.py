"""The allocation-free triangular solve (chol_trisolve_noalloc: workspace in the
library's static device scratch) against chol_trisolve, the entry point it is
a variant of, through the C ABI.  Both run the same kernels in the same order,
so the solutions must agree bit for bit; each is also checked against the
oracle's substitution (relative forward error <= 1e-13 in binary64, <= 2e-5 in
binary32).  Two calls in a row, the second smaller, show that what the scratch
keeps from a call does not leak into the next."""
import numpy as np
import pytest

import oracle
from paper_1812_02056_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1812_02056_amd import binding  # noqa: E402

DEV = torch.device("cuda:0")
STORE = {"f64": torch.float64, "f32": torch.float32}
TOL = {"f64": 1e-13, "f32": 2e-5}


def solve_both(n, nrhs, dtype, seed):
    A = wl.spd_scaled(n, seed=seed)
    Lo, info = oracle.chol(A)
    assert info == 0
    B = wl.rhs(n, nrhs, seed=seed + 1)
    st = STORE[dtype]
    L = binding.to_device(Lo, DEV, dtype=st, ld=n + 3)
    X1 = binding.to_device(B, DEV, dtype=st, ld=n + 1)
    X2 = binding.to_device(B, DEV, dtype=st, ld=n + 1)
    binding.chol_trisolve(L, X1, dtype=dtype)
    status = torch.full((1,), 7, dtype=torch.int32, device=DEV)
    binding.chol_trisolve_noalloc(L, X2, dtype=dtype, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    assert torch.equal(X1, X2)
    Xo = oracle.chol_solve(Lo, B)
    assert oracle.fwd_x(X2.cpu().numpy().astype(np.float64), Xo) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_matches_chol_trisolve_two_calls(dtype):
    solve_both(3000, 5, dtype, seed=51)
    solve_both(1100, 2, dtype, seed=53)      # smaller, right after


def test_noalloc_largest_binary64_size():
    solve_both(9344, 1, "f64", seed=55)


def test_noalloc_empty_rhs_sets_status():
    L = binding.to_device(np.eye(8), DEV)
    X = binding.colmajor_empty(8, 0, torch.float64, DEV)
    status = torch.full((1,), 7, dtype=torch.int32, device=DEV)
    binding.chol_trisolve_noalloc(L, X, dtype="f64", status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
