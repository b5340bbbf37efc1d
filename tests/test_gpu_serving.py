"""GPU tests of the serving path (ff_server_*): many independent SPD systems
factored together with grouped launches, through the C ABI.

Each request must give exactly the result of the single-matrix path with the
same step size: the grouped launches run the same per-block kernels (diagonal
factorisation, panel solve) and the same per-tile update body with the same
accumulation order, so the factor and the solution are bitwise equal to
chol_factor + chol_trisolve on the request alone (binary64 server), or to
chol_solve with a binary32 factor, refinement tolerance 1e-12 and at most 30
iterations (binary32 server: the same refinement kernels and the same stop
rule, so also the same iteration count).  Against the oracle the tolerances are
those of the binary64 path (fwd_x <= 1e-12 at kappa ~ 5, bitwise on the integer
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


def dev(a):
    return ff.to_device(a, DEV, dtype=torch.float64)


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def alone(A, B):
    """The single-matrix path with the server's step size (192 columns, at most n)."""
    n = A.shape[0]
    s = min(n, 192)
    Ad = dev(A)
    info = ff.chol_factor(Ad, s, sync=True)
    X = dev(B)
    ff.chol_trisolve(Ad, X)
    torch.cuda.synchronize()
    return host(X), info


def alone_f32(A, B):
    """The single-matrix binary32 + refinement path with the server's step and stop rule."""
    n = A.shape[0]
    X, _, info = ff.chol_solve(dev(A), dev(B), min(n, 192), dtype="f32", tol=1e-12, max_iter=30)
    torch.cuda.synchronize()
    return host(X), info


def drain(srv, limit=100000):
    out = {}
    for _ in range(limit):
        left = srv.step()
        for r in srv.poll():
            out[r["id"]] = r
        if left == 0:
            break
    torch.cuda.synchronize()
    # poll hands out at most max_out results per call: collect until none is left
    while True:
        got = srv.poll()
        if not got:
            break
        for r in got:
            out[r["id"]] = r
    return out


def arena(nbytes):
    return torch.empty(nbytes // 8 + 1, dtype=torch.float64, device=DEV)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_server_mix_matches_single_path_bitwise(dtype):
    sizes = [64, 300, 513, 129, 1000, 256, 777]
    reqs = []
    srv = ff.Server(arena(1 << 30), dtype=dtype)
    for i, n in enumerate(sizes):
        A = wl.spd_scaled(n, seed=100 + i)
        B = wl.rhs(n, 1 + i % 5, seed=200 + i)
        Ad, Bd = dev(A), dev(B)
        Xd = torch.zeros_like(Bd)
        rid = srv.submit(Ad, Bd, Xd, key=1000 + i)
        reqs.append((rid, A, B, Xd))
    done = drain(srv)
    assert len(done) == len(sizes)
    for rid, A, B, Xd in reqs:
        assert done[rid]["info"] == 0
        assert not done[rid]["cache_hit"]
        if dtype == "f64":
            Xa, info = alone(A, B)
            assert info == 0
        else:
            Xa, sinfo = alone_f32(A, B)
            assert sinfo["info"] == 0
            assert done[rid]["iters"] == sinfo["iters"] and done[rid]["converged"] == bool(sinfo["converged"])
            assert done[rid]["converged"]
        assert np.array_equal(host(Xd), Xa), rid
        Lo, _ = oracle.chol(A)
        assert oracle.fwd_x(host(Xd), oracle.chol_solve(Lo, B)) <= 1e-12
    st = srv.stats()
    assert st["completed"] == len(sizes) and st["resident_factors"] == len(sizes)
    srv.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_server_repeat_key_is_a_cache_hit(dtype):
    n = 640
    A = wl.spd_scaled(n, seed=7)
    Ad = dev(A)
    srv = ff.Server(arena(1 << 28), dtype=dtype)
    B1, B2 = wl.rhs(n, 3, seed=8), wl.rhs(n, 2, seed=9)
    B1d = dev(B1)
    X1 = torch.zeros_like(B1d)
    r1 = srv.submit(Ad, B1d, X1, key=42)
    d1 = drain(srv)
    # the same key again: served from the resident factor, no factorisation
    B2d = dev(B2)
    X2 = torch.zeros_like(B2d)
    r2 = srv.submit(Ad, B2d, X2, key=42)
    steps_before = srv.stats()["grouped_launches"]
    d2 = drain(srv)
    assert d1[r1]["info"] == 0 and not d1[r1]["cache_hit"]
    assert d2[r2]["info"] == 0 and d2[r2]["cache_hit"]
    assert srv.stats()["grouped_launches"] == steps_before      # no block step ran for the hit
    Xa, _ = alone(A, B2) if dtype == "f64" else alone_f32(A, B2)
    assert np.array_equal(host(X2), Xa)
    srv.close()


def test_server_f32_mixed_sizes_and_conditioning_against_oracle():
    # binary32 factors refined in binary64: every result within the binary64 tolerance
    srv = ff.Server(arena(1 << 30), dtype="f32")
    cases = []
    for i, (n, lam) in enumerate(((333, 1.0), (700, 1e-2), (1024, 1e-3), (95, 1.0))):
        A = wl.spd_scaled(n, seed=80 + i, lam=lam)
        B = wl.rhs(n, 1 + i, seed=90 + i)
        Bd = dev(B)
        Xd = torch.zeros_like(Bd)
        cases.append((srv.submit(dev(A), Bd, Xd, key=300 + i), A, B, Xd))
    done = drain(srv)
    for rid, A, B, Xd in cases:
        assert done[rid]["info"] == 0 and done[rid]["iters"] >= 1
        Lo, _ = oracle.chol(A)
        Xo = oracle.chol_solve(Lo, B)
        assert oracle.bwd_x(A, host(Xd), B) <= 1e-15
        assert oracle.fwd_x(host(Xd), Xo) <= 1e-12
    srv.close()


def test_server_bf16_is_not_served():
    with pytest.raises(ff.FastFactError):
        ff.Server(arena(1 << 20), dtype="bf16")


def test_server_non_spd_reports_info_and_spares_the_others():
    L0, A = wl.chol_int_family(200, seed=21)
    A[133, 133] -= L0[133, 133] ** 2 + 1.0
    good = wl.spd_scaled(300, seed=22)
    srv = ff.Server(arena(1 << 28))
    Bb, Bg = dev(wl.rhs(200, 1, 23)), dev(wl.rhs(300, 2, 24))
    Xb, Xg = torch.zeros_like(Bb), torch.zeros_like(Bg)
    rb = srv.submit(dev(A), Bb, Xb, key=5)
    rg = srv.submit(dev(good), Bg, Xg, key=6)
    done = drain(srv)
    assert done[rb]["info"] == 134
    assert done[rg]["info"] == 0
    Xa, _ = alone(good, wl.rhs(300, 2, 24))
    assert np.array_equal(host(Xg), Xa)
    # a failed factor is not kept: the same key factors again (and fails again)
    Xb2 = torch.zeros_like(Bb)
    rb2 = srv.submit(dev(A), Bb, Xb2, key=5)
    d2 = drain(srv)
    assert d2[rb2]["info"] == 134 and not d2[rb2]["cache_hit"]
    srv.close()


def test_server_integer_family_exact():
    srv = ff.Server(arena(1 << 28))
    cases = []
    for i, n in enumerate((50, 257, 400)):
        L0, A = wl.chol_int_family(n, seed=30 + i)
        x0 = np.random.default_rng(40 + i).integers(-1, 2, size=(n, 2)).astype(np.float64)
        Bd = dev(A @ x0)
        Xd = torch.zeros_like(Bd)
        cases.append((srv.submit(dev(A), Bd, Xd), x0, Xd))
    done = drain(srv)
    for rid, x0, Xd in cases:
        assert done[rid]["info"] == 0
        assert np.array_equal(host(Xd), x0)
    srv.close()


def test_server_evicts_least_recently_used_factors():
    n = 512
    fbytes = n * n * 8
    srv = ff.Server(arena(3 * fbytes))          # room for two factors and the solve workspaces
    mats = [wl.spd_scaled(n, seed=50 + i) for i in range(3)]
    outs = []
    for i, A in enumerate(mats):
        Bd = dev(wl.rhs(n, 1, seed=60 + i))
        Xd = torch.zeros_like(Bd)
        outs.append((srv.submit(dev(A), Bd, Xd, key=70 + i), A, Xd, i))
        drain(srv)
    st = srv.stats()
    assert st["evictions"] >= 1 and st["resident_factors"] <= 2
    # key 70 was evicted first: asking again refactors and is still exact
    Bd = dev(wl.rhs(n, 1, seed=60))
    Xd = torch.zeros_like(Bd)
    rid = srv.submit(dev(mats[0]), Bd, Xd, key=70)
    d = drain(srv)
    assert d[rid]["info"] == 0 and not d[rid]["cache_hit"]
    Xa, _ = alone(mats[0], wl.rhs(n, 1, seed=60))
    assert np.array_equal(host(Xd), Xa)
    srv.close()


def test_server_rejects_requests_that_can_never_fit():
    srv = ff.Server(arena(1 << 20))
    A = dev(wl.spd_scaled(512, seed=1))
    B = dev(wl.rhs(512, 1, 2))
    with pytest.raises(ff.FastFactError):
        srv.submit(A, B, torch.zeros_like(B))
    srv.close()


def test_server_many_small_keyed_requests_all_complete():
    # more distinct resident factors than requests in flight: admission must never stall
    srv = ff.Server(arena(1 << 28))
    A = wl.spd_scaled(40, seed=3)
    Ad = dev(A)
    B = dev(wl.rhs(40, 1, 4))
    outs = []
    for i in range(700):
        X = torch.zeros_like(B)
        outs.append((srv.submit(Ad, B, X, key=10_000 + i), X))
    done = drain(srv)
    assert len(done) == 700 and all(r["info"] == 0 for r in done.values())
    Xa, _ = alone(A, wl.rhs(40, 1, 4))
    assert all(np.array_equal(host(X), Xa) for _, X in outs[::97])
    srv.close()
